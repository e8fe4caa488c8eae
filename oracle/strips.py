"""Oracle: strip expansions of infinite uniform square-lattice networks (Sec. IV.C).

TEST INFRASTRUCTURE ONLY (see package docstring).  FP64 throughout.

The lattice repeats one tensor A[l, r, u, d] over the legs (-x, +x, -y, +y).
Its BP fixed point is translation invariant: four messages mL, mR, mU, mD,
the ones arriving on a site's -x, +x, -y and +y legs.  The rank-1 projector of
a horizontal bond is P = mR mL^T / n_h with n_h = mR . mL (the message
arriving at the left site's +x leg times the one arriving at the right
site's -x leg), and likewise n_v = mD . mU vertically (Eq. (8) in the
oblique form).

A partition is the set of horizontal bonds (vertical partition lines) that
cross every L-th column line at one offset, or the vertical bonds crossing
every L-th row line.  Inserting P on a partition cuts the lattice into strips;
on two crossing partitions into finite patches.  Per unit cell (L columns, or
L x L sites):

* lam_hat[k]   leading eigenvalue of the width-k vertical transfer matrix
               (k sites in a row, outer legs capped by mL and mR, the k-1
               inner bonds summed), divided by n_h (one cut bond per row);
* gam_hat[k]   the same for width-k horizontal strips, divided by n_v;
* patch_hat[k][p]  the k x p patch (k columns, p rows) with every outer leg
               capped by its arriving message, divided by n_v^k n_h^p.

The combinatorial form (Eq. (7)) over the L vertical (and L horizontal)
partitions, taken per unit cell as the paper does, gives

  1D: f = -(1/L)   log sum_{xv != 0} (-1)^(|xv|+1) prod_{gaps g of xv} lam_hat[g]
  2D: f = -(1/L^2) log sum_{(xv, xh) != 0} (-1)^(|xv|+|xh|+1) W(xv, xh)

with W = prod_g lam_hat[g]^L when xh is empty, prod_g gam_hat[g]^L when xv is
empty, and prod_{gv, gh} patch_hat[gv][gh] otherwise; the gaps of a set of
offsets are the cyclic distances between consecutive offsets (L for one).
For L = 2 these are the paper's width-2 formulas.  f is per lattice site
(per tensor).

Parity pins (tests): the Ising strip eigenvalues against the spin-basis
transfer matrix of a free-boundary strip, Ising patches against brute-force
spin sums, BP exactness on width-one strips, exactness for product tensors,
the paper's L = 2 formulas, and Onsager's free energy as the widths grow.
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def uniform_bp(A, tol=1e-14, max_iter=10000):
    """Jacobi BP on the infinite lattice: (mL, mR, mU, mD, iterations)."""
    chi_h, chi_v = A.shape[0], A.shape[2]
    mL = np.ones(chi_h) / math.sqrt(chi_h)
    mR = mL.copy()
    mU = np.ones(chi_v) / math.sqrt(chi_v)
    mD = mU.copy()

    def norm(v):
        v = v / np.linalg.norm(v)
        return -v if v.sum() < 0 else v

    for it in range(1, max_iter + 1):
        # the message arriving on a -x leg is what the left neighbour sends
        # out of its +x leg: A contracted with its own -x, -y, +y arrivals
        nL = norm(np.einsum("lrud,l,u,d->r", A, mL, mU, mD))
        nR = norm(np.einsum("lrud,r,u,d->l", A, mR, mU, mD))
        nU = norm(np.einsum("lrud,l,r,u->d", A, mL, mR, mU))
        nD = norm(np.einsum("lrud,l,r,d->u", A, mL, mR, mD))
        res = max(np.abs(nL - mL).max(), np.abs(nR - mR).max(), np.abs(nU - mU).max(), np.abs(nD - mD).max())
        mL, mR, mU, mD = nL, nR, nU, nD
        if res <= tol:
            return mL, mR, mU, mD, it
    return mL, mR, mU, mD, max_iter


def overlaps(m):
    mL, mR, mU, mD = m[:4]
    return float(mR @ mL), float(mD @ mU)


def bp_site_weight(A, m):
    """z / (n_h n_v): the BP value per site."""
    mL, mR, mU, mD = m[:4]
    z = float(np.einsum("lrud,l,r,u,d->", A, mL, mR, mU, mD))
    n_h, n_v = overlaps(m)
    return z / (n_h * n_v)


def vertical_transfer(A, m, k):
    """Dense width-k transfer matrix T[(u_1..u_k), (d_1..d_k)]."""
    mL, mR = m[0], m[1]
    chi_v = A.shape[2]
    # R[h, U, D]: the row so far, open right leg h
    R = np.einsum("l,lrud->rud", mL, A).reshape(A.shape[1], chi_v, chi_v)
    for _ in range(1, k):
        R = np.einsum("hUD,hrud->rUuDd", R, A)
        R = R.reshape(A.shape[1], R.shape[1] * chi_v, R.shape[3] * chi_v)
    return np.einsum("hUD,h->UD", R, mR)


def _rotate(A):
    """The lattice seen with x and y exchanged: legs (-y, +y, -x, +x)."""
    return np.ascontiguousarray(A.transpose(2, 3, 0, 1))


def _leading(T):
    ev = np.linalg.eigvals(T)
    return float(ev[np.argmax(np.abs(ev))].real)


def lam_hat(A, m, k):
    n_h, _ = overlaps(m)
    return _leading(vertical_transfer(A, m, k)) / n_h


def gam_hat(A, m, k):
    mL, mR, mU, mD = m[:4]
    _, n_v = overlaps(m)
    return _leading(vertical_transfer(_rotate(A), (mU, mD, mL, mR), k)) / n_v


def patch_hat(A, m, k, p):
    """The k x p patch, outer legs capped, by rows of dense transfer matrices."""
    mL, mR, mU, mD = m[:4]
    n_h, n_v = overlaps(m)
    T = vertical_transfer(A, m, k)
    top = mU
    bot = mD
    for _ in range(1, k):
        top = np.kron(top, mU)
        bot = np.kron(bot, mD)
    v = top
    log_s = 0.0
    for _ in range(p):
        v = v @ T
        s = float(np.abs(v).max())
        v = v / s
        log_s += math.log(s)
    return float(v @ bot) * math.exp(log_s) / (n_v ** k * n_h ** p)


def gaps(x, L):
    """Cyclic distances between consecutive offsets of x (sorted); [L] for one."""
    x = sorted(x)
    return [((x[(i + 1) % len(x)] - x[i] - 1) % L) + 1 for i in range(len(x))]


def strip_combination(lam, gam, patch, L, two_d=True):
    """The per-cell sum of Eq. (7) over the strip partitions (lam, gam indexed
    1..L, patch[k][p]); returns the free energy per site."""
    total = 0.0
    offs = range(L)
    subsets = [x for r in range(L + 1) for x in itertools.combinations(offs, r)]
    for xv in subsets:
        for xh in (subsets if two_d else [()]):
            if not xv and not xh:
                continue
            sgn = 1.0 if (len(xv) + len(xh)) % 2 == 1 else -1.0
            if not xh:
                w = math.prod(lam[g] for g in gaps(xv, L)) ** (L if two_d else 1)
            elif not xv:
                w = math.prod(gam[g] for g in gaps(xh, L)) ** L
            else:
                w = math.prod(patch[gv][gh] for gv in gaps(xv, L) for gh in gaps(xh, L))
            total += sgn * w
    return -math.log(total) / (L * L if two_d else L)


def strip_expansion(A, L, two_d=True, m=None):
    """Every quantity of the width-L strip expansion and the free energy."""
    if m is None:
        m = uniform_bp(A)
    lam = {k: lam_hat(A, m, k) for k in range(1, L + 1)}
    gam = {k: gam_hat(A, m, k) for k in range(1, L + 1)} if two_d else {}
    patch = {k: {p: patch_hat(A, m, k, p) for p in range(1, L + 1)} for k in range(1, L + 1)} if two_d else {}
    f = strip_combination(lam, gam, patch, L, two_d)
    return {"lam": lam, "gam": gam, "patch": patch, "f": f, "f_bp": -math.log(bp_site_weight(A, m)), "m": m}


def onsager_f(beta):
    """-ln Z / N of the infinite 2D Ising model (J = 1), Onsager's solution in
    its single-integral form."""
    from scipy.integrate import quad

    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2

    def integrand(t):
        return math.log(0.5 * (1.0 + math.sqrt(max(0.0, 1.0 - (k * math.sin(t)) ** 2))))

    val, _ = quad(integrand, 0.0, math.pi / 2, epsabs=1e-14, epsrel=1e-14, limit=200)
    return -(math.log(2.0 * math.cosh(2 * beta)) + val / math.pi)
