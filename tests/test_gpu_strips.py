"""GPU parity for the infinite-lattice strip expansion (Sec. IV.C).

The HIP path (uniform BP, power iteration of every strip transfer matrix,
patches, cell sum) against the oracle's dense transfer matrices and exact
patches, at widths the oracle finishes in seconds; at the full width (L = 12,
the benchmark's size) sampled strips against spin-basis transfer matrices and
dense oracle strips, and the free energy against Onsager's solution.

Tolerances: the ratios lam_k / w^k, gam_k / w^k and Z_kp / w^(kp) to 1e-11
relative (power iteration stops at 1e-13 relative change); f to 1e-12
absolute.
"""

import math

import numpy as np
import pytest

import pne_inputs as P
from oracle import strips as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_10910_amd as pne

    c = pne.Context(0)
    yield c
    c.close()


CASES = [
    ("ising_b0.3", lambda: P.ising_uniform_tensor(0.3), 5),
    ("ising_b0.4407", lambda: P.ising_uniform_tensor(0.4407), 5),
    ("ising_b0.6", lambda: P.ising_uniform_tensor(0.6), 5),
    ("blocked_ising_b0.3", lambda: P.ising_blocked_tensor(0.3), 3),
    ("blocked_ising_b0.4407", lambda: P.ising_blocked_tensor(0.4407), 3),
    ("random_chi3", lambda: P.random_uniform_tensor(3, seed=7, bias=1.0), 4),
    ("random_chi5", lambda: P.random_uniform_tensor(5, seed=8, bias=1.0), 2),
    ("random_chi6", lambda: P.random_uniform_tensor(6, seed=9, bias=1.0), 2),
]


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("single_site", [False, True])
@pytest.mark.parametrize("name,make,L", CASES)
def test_strip_expansion_matches_oracle(ctx, name, make, L, single_site):
    """Both pass layouts: two neighbouring sites per pass (chi <= 4, the
    default) and one site per pass."""
    A = make()
    r = ctx.strip_expand(A, L, single_site_passes=single_site)
    ref = S.strip_expansion(A, L)
    w = math.exp(-ref["f_bp"])
    print(name, r["f"], ref["f"], r["power_iters"], flush=True)
    assert r["status"] == 0 and r["n_unconverged"] == 0
    assert abs(r["f_bp"] - ref["f_bp"]) < 1e-13
    for k in range(1, L + 1):
        assert _rel(r["lam_ratio"][k - 1], ref["lam"][k] / w ** k) < 1e-11, ("lam", k)
        assert _rel(r["gam_ratio"][k - 1], ref["gam"][k] / w ** k) < 1e-11, ("gam", k)
        for p in range(1, L + 1):
            assert _rel(r["patch_ratio"][k - 1, p - 1], ref["patch"][k][p] / w ** (k * p)) < 1e-11, ("patch", k, p)
    assert abs(r["f"] - ref["f"]) < 1e-12


def test_vertical_strips_only(ctx):
    A = P.ising_uniform_tensor(0.5)
    r = ctx.strip_expand(A, 4, two_d=False)
    ref = S.strip_expansion(A, 4, two_d=False)
    assert abs(r["f"] - ref["f"]) < 1e-12


def test_blocked_ising_full_width(ctx):
    """The benchmark's size: 2 x 2-blocked Ising (chi = 4), width-12 strips in
    both directions.  Strips up to width 5 against dense oracle transfer
    matrices, patches up to 3 x 3 against exact patches, and the free energy
    per spin against Onsager (closer than at width 3)."""
    beta = 0.3
    A = P.ising_blocked_tensor(beta)
    r = ctx.strip_expand(A, 12)
    r1 = ctx.strip_expand(A, 12, single_site_passes=True)
    assert abs(r["f"] - r1["f"]) < 1e-13
    assert r["status"] == 0 and r["n_unconverged"] == 0
    m = S.uniform_bp(A)
    w = S.bp_site_weight(A, m)
    for k in range(1, 6):
        assert _rel(r["lam_ratio"][k - 1], S.lam_hat(A, m, k) / w ** k) < 1e-11, k
        assert _rel(r["gam_ratio"][k - 1], S.gam_hat(A, m, k) / w ** k) < 1e-11, k
    for k in (1, 2, 3):
        for p in (1, 2, 3, 12):
            assert _rel(r["patch_ratio"][k - 1, p - 1], S.patch_hat(A, m, k, p) / w ** (k * p)) < 1e-11, (k, p)
    exact = S.onsager_f(beta)
    err12 = abs(r["f"] / 4 - exact)
    err3 = abs(S.strip_expansion(A, 3, m=m)["f"] / 4 - exact)
    print("L=12 error per spin", err12, "L=3", err3, flush=True)
    assert err12 < err3 and err12 < 1e-9


def test_strip_errors(ctx):
    import paper_2512_10910_amd as pne

    with pytest.raises(pne.PNEError) as e:
        ctx.strip_expand(np.ones((7, 7, 7, 7)), 2)
    assert e.value.status == -2
    with pytest.raises(pne.PNEError) as e:
        ctx.strip_expand(np.ones((2, 2, 2, 2)), 0)
    assert e.value.status == -1
    bad = np.ones((2, 2, 2, 2))
    bad[0, 0, 0, 0] = np.nan
    with pytest.raises(pne.PNEError) as e:
        ctx.strip_expand(bad, 2)
    assert e.value.status == -1
    with pytest.raises(pne.PNEError) as e:
        ctx.strip_expand(np.ones((4, 4, 4, 4)), 16)
    assert e.value.status == -2
