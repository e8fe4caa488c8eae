"""Pins of the strip-expansion oracle (infinite lattices, Sec. IV.C).

Independent of the oracle's own construction: Ising strips and patches from
the spin basis (transfer matrices with exp(beta s s') bond weights, brute
force spin sums), BP exactness on width-one strips (a chain), exactness for
product tensors, the paper's printed width-2 formulas, and Onsager's free
energy (checked itself at the critical point against Catalan's constant).
"""

import itertools
import math

import numpy as np
import pytest

import pne_inputs as P
from oracle import strips as S

BETAS = [0.3, 0.4, 0.6]


def _spin_strip_matrix(beta, w):
    """Row-to-row transfer matrix of a width-w free-boundary Ising strip,
    symmetrised: D^1/2 B D^1/2 with B the vertical bond weights and D the
    row's own horizontal bond weights."""
    states = np.array(list(itertools.product((1, -1), repeat=w)))
    B = np.exp(beta * states @ states.T)
    h = np.exp(beta * (states[:, :-1] * states[:, 1:]).sum(axis=1)) if w > 1 else np.ones(len(states))
    d = np.sqrt(h)
    return d[:, None] * B * d[None, :], h


def _spin_lam(beta, w):
    V, _ = _spin_strip_matrix(beta, w)
    return float(np.linalg.eigvalsh(V)[-1])


def _spin_patch(beta, w, rows):
    """Free-boundary Ising partition function of a w-wide, rows-tall patch."""
    states = np.array(list(itertools.product((1, -1), repeat=w)))
    B = np.exp(beta * states @ states.T)
    h = np.exp(beta * (states[:, :-1] * states[:, 1:]).sum(axis=1)) if w > 1 else np.ones(len(states))
    v = h.copy()
    for _ in range(rows - 1):
        v = (v @ B) * h
    return float(v.sum())


def test_onsager_at_the_critical_point():
    catalan = 0.915965594177219015054603514932
    bc = 0.5 * math.log(1 + math.sqrt(2))
    assert abs(S.onsager_f(bc) + (0.5 * math.log(2) + 2 * catalan / math.pi)) < 1e-12


@pytest.mark.parametrize("beta", BETAS)
def test_ising_strip_eigenvalues_match_the_spin_basis(beta):
    """Each cap contributes sqrt(cosh beta) (W applied to the uniform
    message), so lam_k = cosh(beta) * (leading eigenvalue of the width-k
    spin transfer matrix)."""
    A = P.ising_uniform_tensor(beta)
    m = S.uniform_bp(A)
    for k in range(1, 6):
        assert abs(S.lam_hat(A, m, k) - math.cosh(beta) * _spin_lam(beta, k)) <= 1e-12 * S.lam_hat(A, m, k)
        assert abs(S.gam_hat(A, m, k) - S.lam_hat(A, m, k)) <= 1e-12 * S.lam_hat(A, m, k)


def _phi(beta, cap):
    """Boundary weight of a capped merged leg on its two spins: the cap
    pushed through the two spin bonds' square roots W."""
    W = P.networks._ising_w(beta)
    c = np.asarray(cap).reshape(2, 2)
    return np.einsum("sa,tb,ab->st", W, W, c)


def _blocked_spin_lam(beta, k, m):
    """Block-row transfer matrix written over spins: 2k spins per spin row,
    two spin rows (r, t) per block row, B between rows, the rows' own
    horizontal bonds, and the side caps acting on (r_first, t_first) and
    (r_last, t_last)."""
    states = np.array(list(itertools.product((1, -1), repeat=2 * k)))
    idx = (1 - states) // 2
    B = np.exp(beta * states @ states.T)
    h = np.exp(beta * (states[:, :-1] * states[:, 1:]).sum(axis=1))
    fl, fr = _phi(beta, m[0]), _phi(beta, m[1])
    side = fl[idx[:, 0][:, None], idx[:, 0][None, :]] * fr[idx[:, -1][:, None], idx[:, -1][None, :]]
    # T[s, t] = sum_r B[s, r] h[r] B[r, t] h[t] side[r, t]
    T = np.einsum("sr,r,rt,t,rt->st", B, h, B, h, side)
    n_h, _ = S.overlaps(m)
    ev = np.linalg.eigvals(T)
    return float(ev[np.argmax(np.abs(ev))].real) / n_h


def _blocked_spin_patch(beta, k, p, m):
    """Brute-force spin sum of the k x p block patch (2k x 2p spins) with
    every outer merged leg capped."""
    Wd, H = 2 * k, 2 * p
    fu, fd, fl, fr = (_phi(beta, m[i]) for i in (2, 3, 0, 1))
    n_h, n_v = S.overlaps(m)
    Z = 0.0
    for spins in itertools.product((1, -1), repeat=Wd * H):
        g = np.array(spins).reshape(H, Wd)
        e = (g[:, :-1] * g[:, 1:]).sum() + (g[:-1, :] * g[1:, :]).sum()
        ix = (1 - g) // 2
        w = math.exp(beta * e)
        for bx in range(k):
            w *= fu[ix[0, 2 * bx], ix[0, 2 * bx + 1]] * fd[ix[H - 1, 2 * bx], ix[H - 1, 2 * bx + 1]]
        for by in range(p):
            w *= fl[ix[2 * by, 0], ix[2 * by + 1, 0]] * fr[ix[2 * by, Wd - 1], ix[2 * by + 1, Wd - 1]]
        Z += w
    return Z / (n_v ** k * n_h ** p)


@pytest.mark.parametrize("beta", BETAS)
def test_blocked_ising_strips_and_patches(beta):
    """The 2 x 2-blocked tensor, with its own (better than per-spin) BP
    messages as caps, against the same strips and patches written over
    spins: width-k block strips as two-row spin transfer matrices, k x p
    block patches as brute-force spin sums."""
    A = P.ising_blocked_tensor(beta)
    m = S.uniform_bp(A)
    for k in (1, 2, 3):
        ref = _blocked_spin_lam(beta, k, m)
        assert abs(S.lam_hat(A, m, k) - ref) <= 1e-11 * ref
    for k, p in ((1, 1), (1, 2), (2, 1), (2, 2)):
        ref = _blocked_spin_patch(beta, k, p, m)
        assert abs(S.patch_hat(A, m, k, p) - ref) <= 1e-11 * ref


@pytest.mark.parametrize("beta", [0.3, 0.5])
def test_ising_patches_against_brute_force(beta):
    A = P.ising_uniform_tensor(beta)
    m = S.uniform_bp(A)
    for k, p in ((1, 1), (2, 1), (2, 3), (3, 3), (4, 2)):
        n = k * p
        Z = 0.0
        for spins in itertools.product((1, -1), repeat=n):
            s = np.array(spins).reshape(p, k)
            e = (s[:, :-1] * s[:, 1:]).sum() + (s[:-1, :] * s[1:, :]).sum()
            Z += math.exp(beta * e)
        ref = Z * math.cosh(beta) ** (k + p)
        assert abs(S.patch_hat(A, m, k, p) - ref) <= 1e-12 * ref


@pytest.mark.parametrize("seed", [1, 2])
def test_width_one_strips_are_exact_for_bp(seed):
    """A width-one strip is a chain, where BP is exact: lam_1, gam_1 and the
    1 x p patches equal the BP value per site (to the power p)."""
    A = P.random_uniform_tensor(3, seed=seed, bias=1.0)
    m = S.uniform_bp(A)
    w = S.bp_site_weight(A, m)
    assert abs(S.lam_hat(A, m, 1) - w) <= 1e-12 * w
    assert abs(S.gam_hat(A, m, 1) - w) <= 1e-12 * w
    for p in (1, 2, 3):
        assert abs(S.patch_hat(A, m, 1, p) - w ** p) <= 1e-12 * w ** p
        assert abs(S.patch_hat(A, m, p, 1) - w ** p) <= 1e-12 * w ** p


def test_product_tensor_is_exact_at_every_width():
    rng = np.random.default_rng(5)
    a, b, c, d = (rng.uniform(0.5, 1.5, 3) for _ in range(4))
    A = np.einsum("l,r,u,d->lrud", a, b, c, d)
    z = float(a @ b) * float(c @ d)
    for L in (1, 2, 3):
        r = S.strip_expansion(A, L)
        assert abs(r["f"] + math.log(z)) < 1e-12
        assert abs(r["f_bp"] + math.log(z)) < 1e-12


def test_the_printed_width_two_and_three_formulas():
    """General-L subset sums reproduce the paper's L = 2 formulas (and the
    L = 3 vertical one, with the sign Eq. (7) gives the pair terms)."""
    rng = np.random.default_rng(3)
    lam = {k: rng.uniform(0.9, 1.1) * 2 ** k for k in (1, 2, 3)}
    gam = {k: rng.uniform(0.9, 1.1) * 2 ** k for k in (1, 2)}
    Z = {k: {p: rng.uniform(0.9, 1.1) * 2 ** (k * p) for p in (1, 2)} for k in (1, 2)}
    f1 = S.strip_combination(lam, {}, {}, 2, two_d=False)
    assert abs(f1 + math.log(2 * lam[2] - lam[1] ** 2) / 2) < 1e-14
    f3 = S.strip_combination(lam, {}, {}, 3, two_d=False)
    assert abs(f3 + math.log(3 * lam[3] - 3 * lam[2] * lam[1] + lam[1] ** 3) / 3) < 1e-14
    R1 = 2 * lam[2] ** 2 + 2 * gam[2] ** 2
    R2 = 4 * Z[2][2] + lam[1] ** 4 + gam[1] ** 4
    R3 = 2 * Z[2][1] ** 2 + 2 * Z[1][2] ** 2
    R4 = Z[1][1] ** 4
    f2 = S.strip_combination(lam, gam, Z, 2, two_d=True)
    assert abs(f2 + math.log(R1 - R2 + R3 - R4) / 4) < 1e-14


@pytest.mark.parametrize("beta,L,bound", [(0.3, 3, 2e-6), (0.6, 3, 1e-7)])
def test_blocked_ising_approaches_onsager(beta, L, bound):
    """Away from the critical point the blocked width-L expansion sits close
    to the exact free energy, and the error falls as L grows."""
    A = P.ising_blocked_tensor(beta)
    m = S.uniform_bp(A)
    exact = S.onsager_f(beta)
    errs = [abs(S.strip_expansion(A, w, m=m)["f"] / 4 - exact) for w in range(1, L + 1)]
    assert errs[-1] < bound
    assert errs[0] > errs[-1]


def test_wrong_gaps_break_the_width_two_formula(monkeypatch):
    lam = {1: 2.0, 2: 4.5}
    good = S.strip_combination(lam, {}, {}, 2, two_d=False)
    assert abs(good + math.log(2 * 4.5 - 4.0) / 2) < 1e-14
    orig = S.gaps
    monkeypatch.setattr(S, "gaps", lambda x, L: [L] * len(x))
    try:
        bad = S.strip_combination(lam, {}, {}, 2, two_d=False)
    except ValueError:  # the mutated sum is not positive
        bad = math.inf
    assert abs(bad - good) > 1e-3
    monkeypatch.setattr(S, "gaps", orig)
