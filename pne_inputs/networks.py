"""Seeded tensor-network constructions (inputs only; no expansion arithmetic).

Conventions shared by every consumer:

* A network is a list of site tensors plus a bond list.  Site ``s`` holds an
  FP64 array in C order over its *leg slots*.
* On lattices, sites are numbered row-major with x fastest
  (``s = x + Lx*y`` in 2D, ``s = x + L*(y + L*z)`` in 3D).  A site's bond legs
  come in the canonical order (-x, +x, -y, +y, -z, +z), keeping only the
  directions that exist under open boundaries; open (physical) legs follow.
* ``bonds[b] = (u, leg_u, v, leg_v)`` joins leg slot ``leg_u`` of site ``u``
  to leg slot ``leg_v`` of site ``v``.  Lattice bonds are listed site by site
  in the order +x, +y, +z.
* ``open_legs[k] = (site, leg)`` lists legs that stay uncontracted.

The physical constructions follow the paper's Appendix A: the Ising partition
function in the usual symmetric-square-root encoding, the AKLT PEPS norm
(physical dimension 5, virtual dimension 2, merged bond dimension 4) and
random tensors with i.i.d. entries.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from functools import reduce

import numpy as np


@dataclass
class Network:
    tensors: list
    bonds: np.ndarray  # (M, 4) int32: u, leg_u, v, leg_v
    open_legs: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    name: str = ""
    info: dict = field(default_factory=dict)

    @property
    def n_sites(self) -> int:
        return len(self.tensors)

    @property
    def n_bonds(self) -> int:
        return int(self.bonds.shape[0])

    @property
    def n_open(self) -> int:
        return int(self.open_legs.shape[0])

    def bond_dim(self, b: int) -> int:
        u, lu, _, _ = self.bonds[b]
        return int(self.tensors[u].shape[lu])

    def nbytes(self) -> int:
        return int(sum(t.nbytes for t in self.tensors))


# ----------------------------------------------------------------------------
# lattice geometry


_DIRS = ("-x", "+x", "-y", "+y", "-z", "+z")


def _lattice(shape):
    """Return (site_dirs, bonds) for an open-boundary hypercubic lattice.

    ``site_dirs[s]`` maps a direction name to the site's leg slot.  Cached
    per shape (callers must not modify the result).
    """
    shape = tuple(int(x) for x in shape)
    hit = _LATTICE_CACHE.get(shape)
    if hit is None:
        site_dirs, bonds = _lattice_uncached(shape)
        bonds.setflags(write=False)  # shared by every network of this shape
        hit = _LATTICE_CACHE[shape] = (site_dirs, bonds)
    return hit


_LATTICE_CACHE = {}


def _lattice_uncached(shape):
    nd = len(shape)
    dims = list(shape)
    n = int(np.prod(dims))
    strides = [int(np.prod(dims[:k])) for k in range(nd)]
    coords = []
    for s in range(n):
        c = []
        r = s
        for k in range(nd):
            c.append(r % dims[k])
            r //= dims[k]
        coords.append(c)
    site_dirs = []
    for s in range(n):
        c = coords[s]
        slots = {}
        for k in range(nd):
            if c[k] > 0:
                slots[_DIRS[2 * k]] = len(slots)
            if c[k] < dims[k] - 1:
                slots[_DIRS[2 * k + 1]] = len(slots)
        site_dirs.append(slots)
    bonds = []
    for s in range(n):
        c = coords[s]
        for k in range(nd):
            if c[k] < dims[k] - 1:
                t = s + strides[k]
                bonds.append((s, site_dirs[s][_DIRS[2 * k + 1]], t, site_dirs[t][_DIRS[2 * k]]))
    return site_dirs, np.asarray(bonds, dtype=np.int32).reshape(-1, 4)


def lattice_2d(Lx: int, Ly: int):
    return _lattice((Lx, Ly))


def lattice_3d(L: int):
    return _lattice((L, L, L))


def _site_index(shape, coord):
    s = 0
    mul = 1
    for k, c in enumerate(coord):
        s += c * mul
        mul *= shape[k]
    return s


def _build(shape, make_tensor, open_sites=None, name=""):
    """Assemble a lattice network; ``make_tensor(s, bond_rank, open_dims)``."""
    site_dirs, bonds = _lattice(shape)
    open_sites = dict(open_sites or {})
    tensors = []
    open_legs = []
    for s, slots in enumerate(site_dirs):
        odims = open_sites.get(s, ())
        if isinstance(odims, int):
            odims = (odims,)
        t = make_tensor(s, len(slots), tuple(odims))
        for k in range(len(odims)):
            open_legs.append((s, len(slots) + k))
        tensors.append(np.ascontiguousarray(t, dtype=np.float64))
    ol = np.asarray(open_legs, dtype=np.int32).reshape(-1, 2)
    return Network(tensors, bonds, ol, name=name, info={"shape": tuple(shape)})


# ----------------------------------------------------------------------------
# Ising (Appendix A.1)


def _ising_w(beta: float, J: float = 1.0) -> np.ndarray:
    """Symmetric square root W of the bond Boltzmann matrix B = W W.

    B[s, s'] = exp(beta*J*s*s') for spins s, s' in {+1, -1}; its eigenvalues
    are 2 cosh(beta J) and 2 sinh(beta J) with eigenvectors (1, 1)/sqrt2 and
    (1, -1)/sqrt2.
    """
    l0 = 2.0 * math.cosh(beta * J)
    l1 = 2.0 * math.sinh(beta * J)
    if l1 < 0:
        raise ValueError("antiferromagnetic coupling needs a complex square root")
    a, b = math.sqrt(l0), math.sqrt(l1)
    return 0.5 * np.array([[a + b, a - b], [a - b, a + b]], dtype=np.float64)


def _ising_site(W: np.ndarray, rank: int) -> np.ndarray:
    """T[a_1..a_r] = sum_s prod_l W[s, a_l] (spin s summed at the site)."""
    if rank == 0:
        return np.array(2.0)
    out = np.zeros((2,) * rank)
    for s in range(2):
        out += reduce(np.multiply.outer, [W[s]] * rank)
    return out


def _ising_maker(W):
    """Site tensors by rank, each built once (sites of equal rank share it)."""
    made = {}

    def make(s, r, o):
        if r not in made:
            made[r] = _ising_site(W, r)
            made[r].setflags(write=False)  # shared by every site of rank r
        return made[r]

    return make


def ising_2d(Lx: int, Ly: int, beta: float, J: float = 1.0) -> Network:
    W = _ising_w(beta, J)
    net = _build((Lx, Ly), _ising_maker(W), name=f"ising2d_{Lx}x{Ly}_b{beta}")
    net.info.update(model="ising", beta=beta, J=J)
    return net


def ising_3d(L: int, beta: float, J: float = 1.0) -> Network:
    W = _ising_w(beta, J)
    net = _build((L, L, L), _ising_maker(W), name=f"ising3d_{L}_b{beta}")
    net.info.update(model="ising", beta=beta, J=J)
    return net


# ----------------------------------------------------------------------------
# random tensors (Appendix A.3)


def _draw(rng, shape, dist):
    if dist in ("uniform01", "uniform"):
        return rng.random(shape)
    if dist == "normal":  # mean 1, sd 0.3
        return rng.normal(1.0, 0.3, shape)
    if isinstance(dist, tuple) and dist[0] == "uniform":
        return rng.uniform(dist[1], dist[2], shape)
    if isinstance(dist, tuple) and dist[0] == "normal":
        return rng.normal(dist[1], dist[2], shape)
    raise ValueError(f"unknown distribution {dist!r}")


def random_2d(Lx, Ly, D, dist="uniform01", seed=0, open_sites=None) -> Network:
    """i.i.d. entries, sites drawn in site order from one PCG64 stream.

    ``open_sites`` maps a site index to its open-leg dimension(s).
    """
    rng = np.random.default_rng(seed)
    net = _build((Lx, Ly), lambda s, r, o: _draw(rng, (D,) * r + o, dist),
                 open_sites=open_sites, name=f"rand2d_{Lx}x{Ly}_D{D}_s{seed}")
    net.info.update(model="random", D=D, dist=dist, seed=seed)
    return net


def random_3d(L, D, dist="uniform01", seed=0, open_sites=None) -> Network:
    rng = np.random.default_rng(seed)
    net = _build((L, L, L), lambda s, r, o: _draw(rng, (D,) * r + o, dist),
                 open_sites=open_sites, name=f"rand3d_{L}_D{D}_s{seed}")
    net.info.update(model="random", D=D, dist=dist, seed=seed)
    return net


# ----------------------------------------------------------------------------
# AKLT norm network (Appendix A.2)


def _aklt_projector() -> np.ndarray:
    """Spin-2 PEPS tensor A[p; l, r, u, d] with virtual spin-1/2 legs.

    The physical state p (0..4) is the normalised symmetric combination of the
    four virtual spins with p of them down; a singlet matrix is absorbed on the
    +x and +y legs so every bond carries exactly one singlet.
    """
    A = np.zeros((5, 2, 2, 2, 2))
    for a in np.ndindex(2, 2, 2, 2):
        p = sum(a)
        A[(p,) + a] = 1.0 / math.sqrt(math.comb(4, p))
    eps = np.array([[0.0, 1.0], [-1.0, 0.0]])
    # leg order (-x, +x, -y, +y): absorb eps on +x (axis 2) and +y (axis 4)
    A = np.einsum("pabcd,bB->paBcd", A, eps)
    A = np.einsum("pabcd,dD->pabcD", A, eps)
    return A


def aklt_2d(Lx: int, Ly: int) -> Network:
    """<psi|psi> for the square-lattice AKLT PEPS, ket/bra legs merged (D=4).

    Merged index = 2*ket + bra.  Boundary directions that have no neighbour are
    capped by the SU(2)-invariant vector vec(I2)/sqrt(2).
    """
    A = _aklt_projector()
    E = np.einsum("pabcd,pABCD->aAbBcCdD", A, A).reshape(4, 4, 4, 4)
    cap = np.array([1.0, 0.0, 0.0, 1.0]) / math.sqrt(2.0)
    site_dirs, _ = _lattice((Lx, Ly))

    def make(s, r, o):
        slots = site_dirs[s]
        T = E
        # contract missing directions from the last axis down to keep order
        for k in range(3, -1, -1):
            if _DIRS[k] not in slots:
                T = np.tensordot(T, cap, axes=([k], [0]))
        return T

    net = _build((Lx, Ly), make, name=f"aklt2d_{Lx}x{Ly}")
    net.info.update(model="aklt")
    return net


# ----------------------------------------------------------------------------
# small non-lattice networks used by tests


def ring_network(mats) -> Network:
    """Closed ring: site i holds M_i[left, right]; Z = Tr(M_0 M_1 ... M_{L-1})."""
    L = len(mats)
    tensors = [np.ascontiguousarray(m, dtype=np.float64) for m in mats]
    bonds = [(i, 1, (i + 1) % L, 0) for i in range(L)]
    return Network(tensors, np.asarray(bonds, np.int32), name=f"ring{L}")


def chain_network(tensors) -> Network:
    """Open chain: first/last tensors are vectors, middle ones matrices."""
    L = len(tensors)
    bonds = []
    for i in range(L - 1):
        bonds.append((i, 0 if i == 0 else 1, i + 1, 0))
    return Network([np.ascontiguousarray(t, np.float64) for t in tensors],
                   np.asarray(bonds, np.int32).reshape(-1, 4), name=f"chain{L}")


def grid_from_tensors(shape, tensor_fn, open_sites=None, name="grid") -> Network:
    """Generic lattice builder: ``tensor_fn(site, bond_rank, open_dims)``."""
    return _build(tuple(shape), tensor_fn, open_sites=open_sites, name=name)


def apply_random_gauge(net: Network, seed: int, scale: float = 0.3) -> Network:
    """Insert G G^-1 on every bond with a random well-conditioned G.

    The contraction value is unchanged; the site tensors (and so the BP
    messages) change, which is what the gauge-invariance checks rely on.
    """
    rng = np.random.default_rng(seed)
    tensors = [t.copy() for t in net.tensors]
    for (u, lu, v, lv) in net.bonds:
        D = tensors[u].shape[lu]
        G = np.eye(D) + scale * rng.standard_normal((D, D))
        Gi = np.linalg.inv(G)
        tu = np.tensordot(tensors[u], G, axes=([lu], [0]))
        tensors[u] = np.ascontiguousarray(np.moveaxis(tu, -1, lu))
        tv = np.tensordot(tensors[v], Gi, axes=([lv], [1]))
        tensors[v] = np.ascontiguousarray(np.moveaxis(tv, -1, lv))
    out = Network(tensors, net.bonds.copy(), net.open_legs.copy(),
                  name=net.name + f"_g{seed}", info=dict(net.info, gauge_seed=seed))
    return out


# ----------------------------------------------------------------------------
# the five benchmark workloads


def config1_network(beta: float = 0.44) -> Network:
    """4x4 open-boundary 2D Ising, J=1, zero field."""
    return ising_2d(4, 4, beta)


def config1_betas(n: int, seed: int = 1) -> np.ndarray:
    """Throughput batch: beta_i = 0.44 (1 + 0.01 u_i), u_i ~ U[-1, 1]."""
    u = np.random.default_rng(seed).uniform(-1.0, 1.0, n)
    return 0.44 * (1.0 + 0.01 * u)


def config2_network(D: int = 4, seed: int = 2000) -> Network:
    """16x16 open-boundary random network, i.i.d. U[0,1] entries."""
    return random_2d(16, 16, D, "uniform01", seed)


def config3_ising_network(beta: float) -> Network:
    """6x6x6 open-boundary 3D Ising."""
    return ising_3d(6, beta)


def config3_aklt_network(gauge_seed=None) -> Network:
    """12x12 AKLT norm network; optional random bond gauge (seed 3000+i)."""
    net = aklt_2d(12, 12)
    if gauge_seed is not None:
        net = apply_random_gauge(net, gauge_seed)
    return net


def config4_request(i: int) -> Network:
    """Serving request i (seed 40000+i): 2D L~U{4..32} or 3D L~U{4..8},
    D~U{2,3,4}, entries U[0,1] or N(1, 0.3^2), each choice with p=1/2."""
    rng = np.random.default_rng(40000 + i)
    is3d = bool(rng.random() < 0.5)
    L = int(rng.integers(4, 9)) if is3d else int(rng.integers(4, 33))
    D = int(rng.integers(2, 5))
    dist = "normal" if rng.random() < 0.5 else "uniform01"
    shape = (L, L, L) if is3d else (L, L)
    net = _build(shape, lambda s, r, o: _draw(rng, (D,) * r, dist),
                 name=f"req{i}_{'3d' if is3d else '2d'}_L{L}_D{D}_{dist}")
    net.info.update(model="random", D=D, dist=dist, L=L, dim=3 if is3d else 2, request=i)
    return net


def config4_arrivals(n: int, rate: float, seed: int = 4) -> np.ndarray:
    """Poisson arrival times (seconds) at ``rate`` requests per second."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    return np.cumsum(gaps)


def config5_network(d: int, L: int = 32, D: int = 6, phys: int = 2) -> Network:
    """32x32 D=6 U[0,1] network with open physical legs (dim 2) at
    A = (x=12, y=15) and B = (x=12+d, y=15); seed 5000+d."""
    a = _site_index((L, L), (12, 15))
    b = _site_index((L, L), (12 + d, 15))
    net = random_2d(L, L, D, "uniform01", 5000 + d, open_sites={a: phys, b: phys})
    net.info.update(open_sites=(a, b), separation=d)
    return net


# ----------------------------------------------------------------------------
# small networks with user partitions (Sec. III.A-C): geometry of the
# double-loop (3 x 2 sites) and 3 x 3 examples and their partition choices


ISING_BETA_C = 0.5 * math.log(1.0 + math.sqrt(2.0))  # critical coupling of the 2D Ising model


def bond_index(net: Network, u: int, v: int) -> int:
    """Index of the bond joining sites u and v."""
    for b, (a, _, c, _) in enumerate(net.bonds):
        if {int(a), int(c)} == {u, v}:
            return b
    raise KeyError((u, v))


def small_network(Lx: int, Ly: int, kind: str = "random", D: int = 4, seed: int = 0,
                  bias: float = 1.0) -> Network:
    """Lx x Ly open-boundary network of one of the paper's three tensor kinds.

    kind "ising": critical 2D Ising (D = 2); "aklt": AKLT PEPS norm (D = 4);
    "random": entries drawn i.i.d. uniform in [-1 + bias, 1 + bias]
    (Appendix A.3) with bond dimension D.
    """
    if kind == "ising":
        return ising_2d(Lx, Ly, ISING_BETA_C)
    if kind == "aklt":
        return aklt_2d(Lx, Ly)
    if kind == "random":
        return random_2d(Lx, Ly, D, dist=("uniform", -1.0 + bias, 1.0 + bias), seed=seed)
    raise ValueError(kind)


def double_loop_partitions(net: Network):
    """The three vertical bonds of the 3 x 2 double loop, one partition each."""
    return [[bond_index(net, x, x + 3)] for x in range(3)]


def grid3_single_partitions(net: Network):
    """Four single-index partitions of the 3 x 3 network: the centre's bonds."""
    return [[bond_index(net, 4, t)] for t in (1, 3, 5, 7)]


def grid3_multi_partitions(net: Network):
    """Six multi-index partitions of the 3 x 3 network (site s = x + 3 y).

    Two vertical lines (between columns 0|1 and 1|2), two horizontal lines
    (between rows 0|1 and 1|2) and two anti-diagonal lines (between the
    diagonals x + y = 1|2 and x + y = 2|3); each transects every bond that
    crosses it.
    """
    def cut(pred):
        return [b for b, (u, _, v, _) in enumerate(net.bonds) if pred(int(u), int(v))]

    def xy(s):
        return s % 3, s // 3

    parts = []
    for c in (0, 1):
        parts.append(cut(lambda u, v, c=c: {xy(u)[0], xy(v)[0]} == {c, c + 1}))
    for r in (0, 1):
        parts.append(cut(lambda u, v, r=r: {xy(u)[1], xy(v)[1]} == {r, r + 1}))
    for d in (1, 2):
        parts.append(cut(lambda u, v, d=d: {sum(xy(u)), sum(xy(v))} == {d, d + 1}))
    return parts


# ----------------------------------------------------------------------------
# uniform tensors of infinite square lattices (Sec. IV.C); legs (-x, +x, -y, +y)


def ising_uniform_tensor(beta: float, J: float = 1.0) -> np.ndarray:
    """One Ising site of the infinite square lattice (bond dimension 2)."""
    return _ising_site(_ising_w(beta, J), 4)


def ising_blocked_tensor(beta: float, J: float = 1.0) -> np.ndarray:
    """2 x 2 block of Ising sites (four spins), bond dimension 4.

    Block sites a (top left), b (top right), c (bottom left), d (bottom
    right), each with legs (-x, +x, -y, +y); the four inner bonds are summed.
    A merged outer leg is 2 * (top or left spin's bond) + (other spin's bond):
    -x = (a, c), +x = (b, d), -y = (a, b), +y = (c, d).
    """
    T = ising_uniform_tensor(beta, J)
    # inner bonds: a.+x = b.-x (p), a.+y = c.-y (q), b.+y = d.-y (s), c.+x = d.-x (t)
    full = np.einsum("Lpuq,pRvs,Mtqe,tNsf->LMRNuvef", T, T, T, T, optimize=True)
    # legs: -x = (L: a, M: c), +x = (R: b, N: d), -y = (u: a, v: b), +y = (e: c, f: d)
    return np.ascontiguousarray(full.reshape(4, 4, 4, 4))


def random_uniform_tensor(chi: int, seed: int = 0, bias: float = 1.0) -> np.ndarray:
    """Uniform tensor with entries i.i.d. uniform in [-1 + bias, 1 + bias]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0 + bias, 1.0 + bias, (chi,) * 4)


def grid3x4_recursive_partitions(net: Network):
    """The 3 x 4 example of recursive partitioning (site s = x + 3 y): three
    horizontal lines (between rows 0|1, 1|2, 2|3) and two vertical lines
    (between columns 0|1, 1|2) as first-level partitions 0..2 and 3..4.  The
    two principal terms that leave a 3 x 3 block whole (the top and bottom
    horizontal cuts) are refined by the six-partition expansion of that
    block.  Returns (partitions, {subset: sub-partitions})."""
    def xy(s):
        return s % 3, s // 3

    def cut(pred):
        return [b for b, (u, _, v, _) in enumerate(net.bonds) if pred(int(u), int(v))]

    parts = []
    for r in (0, 1, 2):
        parts.append(cut(lambda u, v, r=r: {xy(u)[1], xy(v)[1]} == {r, r + 1}))
    for c in (0, 1):
        parts.append(cut(lambda u, v, c=c: {xy(u)[0], xy(v)[0]} == {c, c + 1}))

    def block_parts(y0):
        inside = lambda u, v: y0 <= xy(u)[1] <= y0 + 2 and y0 <= xy(v)[1] <= y0 + 2
        sub = []
        for c in (0, 1):
            sub.append(cut(lambda u, v, c=c: inside(u, v) and {xy(u)[0], xy(v)[0]} == {c, c + 1}))
        for r in (0, 1):
            sub.append(cut(lambda u, v, r=r: inside(u, v) and {xy(u)[1] - y0, xy(v)[1] - y0} == {r, r + 1}))
        for d in (1, 2):
            sub.append(cut(lambda u, v, d=d: inside(u, v)
                           and {xy(u)[0] + xy(u)[1] - y0, xy(v)[0] + xy(v)[1] - y0} == {d, d + 1}))
        return sub

    # cutting between rows 0|1 leaves rows 1..3 whole; between rows 2|3, rows 0..2
    return parts, {(0,): block_parts(1), (2,): block_parts(0)}


def block_lattice(net: Network, Lx: int, Ly: int, b: int) -> Network:
    """Group b x b blocks of an Lx x Ly lattice network (site s = x + Lx y,
    canonical legs) into one site each, merging the b parallel legs that
    leave a block on one side into one leg (the first of them most
    significant).  Only exact contraction of the block's inner bonds: an
    input construction (the paper coarse-grains Ising lattices this way)."""
    assert Lx % b == 0 and Ly % b == 0
    site_dirs, _ = _lattice((Lx, Ly))
    BX, BY = Lx // b, Ly // b
    bdirs, _ = _lattice((BX, BY))
    tensors = []
    for by in range(BY):
        for bx in range(BX):
            sites = [(bx * b + i) + Lx * (by * b + j) for j in range(b) for i in range(b)]
            letters = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")
            bond_lab = {}
            ops, subs = [], []
            for s in sites:
                x, y = s % Lx, s // Lx
                lab = []
                for d, slot in sorted(site_dirs[s].items(), key=lambda kv: kv[1]):
                    nx, ny = x + (d == "+x") - (d == "-x"), y + (d == "+y") - (d == "-y")
                    key = tuple(sorted([(x, y), (nx, ny)]))
                    if key not in bond_lab:
                        bond_lab[key] = next(letters)
                    lab.append(bond_lab[key])
                ops.append(net.tensors[s])
                subs.append("".join(lab))
            # outer legs per direction, ordered along the side
            groups = {}
            for s in sites:
                x, y = s % Lx, s // Lx
                for d in site_dirs[s]:
                    nx, ny = x + (d == "+x") - (d == "-x"), y + (d == "+y") - (d == "-y")
                    if nx // b == bx and ny // b == by:
                        continue
                    key = tuple(sorted([(x, y), (nx, ny)]))
                    pos = y if d in ("-x", "+x") else x
                    groups.setdefault(d, []).append((pos, bond_lab[key]))
            out = []
            for d in _DIRS[:4]:
                if d in bdirs[bx + BX * by]:
                    out.extend(l for _, l in sorted(groups[d]))
            T = np.einsum(",".join(subs) + "->" + "".join(out), *ops, optimize=True)
            shape = []
            k = 0
            for d in _DIRS[:4]:
                if d in bdirs[bx + BX * by]:
                    m = len(groups[d])
                    shape.append(int(np.prod(T.shape[k:k + m])))
                    k += m
            tensors.append(np.ascontiguousarray(T.reshape(shape)))
    _, bonds = _lattice((BX, BY))
    out = Network(tensors, bonds, name=f"{net.name}_blocked{b}", info={"shape": (BX, BY)})
    return out


def ising_blocked_lattice(L: int, b: int, beta: float) -> Network:
    """The L x L open Ising lattice coarse-grained into (L/b) x (L/b) blocks of
    b x b spins (bond dimension 2^b)."""
    net = block_lattice(ising_2d(L, L, beta), L, L, b)
    net.info.update(model="ising", beta=beta, spins=L * L)
    return net
