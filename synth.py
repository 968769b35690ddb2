"""Seeded synthetic inputs for the deterministic neural-backflow NQS hot path.

This module is the ONLY code shared by the FP64 oracle and the HIP path.  It draws
random numbers and lays out arrays; it holds none of the method's arithmetic (no
Hamiltonian matrix element, no network evaluation, no energy).

What it produces
----------------
* One- and two-electron integrals standing in for the RHF/FCIDUMP integrals the
  paper reads (Sec. 3.3, Algorithm 1 input): ``h`` symmetric, diagonal ~ U(-3,-0.5),
  off-diagonal ~ N(0, 0.1^2); ``eri[p,q,r,s] = (pq|rs) = sum_k L^k_pq L^k_rs`` with
  symmetric ``L^k`` ~ N(0, 0.15^2), so the ERI has 8-fold symmetry and is PSD as a
  (pq)x(rs) matrix.  Optionally the off-diagonal parts of ``h`` and ``L^k`` decay as
  exp(-d_pq / xi) for orbitals placed on a 2-D lattice.
* Determinants as ``uint64[n, 2] = (alpha string, beta string)``, bit p = spatial
  orbital p.  Spin-orbital index: alpha p -> p, beta p -> M + p.
* A variational set S: the reference determinant plus excitations of it, filled
  rank by rank (all singles, all doubles, then random triples/quadruples), as a
  stand-in for the top-|psi| selection of a random-init run (Sec. 2.4: V_0 is the
  HF determinant and V grows by selection from its connected set).
* Network parameters theta, packed flat as [W1 b1 W2 b2 ... WL bL Phi0] in
  float32 (W_l row-major d_{l-1} x d_l; Phi0 row-major N_o x N_e), with
  Glorot-uniform weights, zero biases and Phi0 = HF occupation columns plus
  N(0, 1e-3^2) noise (Sec. 3.3).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------- configs
@dataclass(frozen=True)
class Workload:
    """One synthetic workload: system shape, integral recipe and network widths."""
    name: str
    M: int                      # spatial orbitals
    n_alpha: int
    n_beta: int
    rank: int                   # ERI factor rank
    hidden: tuple               # hidden widths
    n_dets: int                 # |S| (0 = full sector)
    lattice: tuple | None = None  # (nx, ny) for 2-D lattice decay, None = no decay
    xi: float = 1.5
    seed: int = 0               # workload index, seeds are derived from it

    @property
    def n_orb(self) -> int:     # N_o, spin orbitals
        return 2 * self.M

    @property
    def n_elec(self) -> int:    # N_e
        return self.n_alpha + self.n_beta

    @property
    def widths(self) -> tuple:
        return (self.n_orb,) + tuple(self.hidden) + (self.n_orb * self.n_elec,)


WORKLOADS = {
    # full 4,900-det sector, tiny MLP
    "m8_4a4b_full": Workload("m8_4a4b_full", 8, 4, 4, 16, (64, 64), 0, seed=1),
    # 16,384 dets in a 1.9e7-det sector
    "m16_5a5b_s16k": Workload("m16_5a5b_s16k", 16, 5, 5, 32, (256, 256), 16384, seed=2),
    # 1e5 dets in a 1.4e12-det sector, lattice-decaying integrals (the headline workload)
    "m28_7a7b_s100k": Workload("m28_7a7b_s100k", 28, 7, 7, 56, (512, 512, 512), 100000,
                               lattice=(7, 4), seed=3),
    # one geometry of the 64-point dissociation curve
    "m20_6a6b_curve": Workload("m20_6a6b_curve", 20, 6, 6, 40, (256, 256), 4096, seed=4),
    # large space, 1e4..1e6 dets
    "m56_12a12b": Workload("m56_12a12b", 56, 12, 12, 112, (1024, 1024), 10000, seed=5),
}


# --------------------------------------------------------------------------- integrals
def make_integrals(M: int, rank: int, seed: int, lattice=None, xi: float = 1.5):
    """Return (h[M,M], eri[M,M,M,M], e_core) as float64 arrays.

    eri is built as sum_k L^k_pq L^k_rs and then symmetrised over the eight index
    permutations so that every symmetry-related element is bit-identical.
    """
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    iu = np.triu_indices(M, 1)
    h[iu] = rng.normal(0.0, 0.1, size=len(iu[0]))
    h = h + h.T
    h[np.diag_indices(M)] = rng.uniform(-3.0, -0.5, size=M)
    L = np.zeros((rank, M, M))
    iu0 = np.triu_indices(M, 0)
    for k in range(rank):
        Lk = np.zeros((M, M))
        Lk[iu0] = rng.normal(0.0, 0.15, size=len(iu0[0]))
        L[k] = Lk + np.triu(Lk, 1).T
    if lattice is not None:
        nx, ny = lattice
        assert nx * ny == M, "lattice must tile the orbitals"
        pos = np.array([(p % nx, p // nx) for p in range(M)], dtype=float)
        d = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
        decay = np.exp(-d / xi)
        np.fill_diagonal(decay, 1.0)
        h = h * decay
        L = L * decay[None]
    Lm = L.reshape(rank, M * M)
    eri = (Lm.T @ Lm).reshape(M, M, M, M)
    eri = symmetrize_eri(eri)
    return h, eri, 0.0


def symmetrize_eri(eri):
    """Average over the 8 real-orbital permutations of (pq|rs)."""
    e = (eri + eri.transpose(1, 0, 2, 3) + eri.transpose(0, 1, 3, 2) + eri.transpose(1, 0, 3, 2)
         + eri.transpose(2, 3, 0, 1) + eri.transpose(3, 2, 0, 1) + eri.transpose(2, 3, 1, 0)
         + eri.transpose(3, 2, 1, 0))
    e = e / 8.0
    # copy each element from its canonical representative so that all eight
    # symmetry-related elements are bit-identical
    M = e.shape[0]
    idx = np.indices((M, M, M, M)).reshape(4, -1).T
    p, q, r, s = idx.T
    a = np.minimum(p, q) * M + np.maximum(p, q)
    b = np.minimum(r, s) * M + np.maximum(r, s)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    cp, cq = lo // M, lo % M
    cr, cs = hi // M, hi % M
    out = e[cp, cq, cr, cs].reshape(M, M, M, M)
    return np.ascontiguousarray(out)


def interpolate_integrals(hA, eriA, hB, eriB, t: float):
    """Convex combination (1-t)A + tB; keeps symmetry and positive semidefiniteness."""
    return (1.0 - t) * hA + t * hB, (1.0 - t) * eriA + t * eriB


# --------------------------------------------------------------------------- determinants
def reference_occupation(h, n_alpha: int, n_beta: int):
    """Occupied spatial orbitals of the reference: lowest diagonal h_pp (stable order)."""
    order = np.argsort(np.diag(h), kind="stable")
    return sorted(order[:n_alpha].tolist()), sorted(order[:n_beta].tolist())


def bits(orbs) -> int:
    v = 0
    for p in orbs:
        v |= 1 << int(p)
    return v


def canonical_sort(dets: np.ndarray) -> np.ndarray:
    """Sort dets lexicographically on (alpha, beta) as unsigned 64-bit integers."""
    dets = np.asarray(dets, dtype=np.uint64).reshape(-1, 2)
    order = np.lexsort((dets[:, 1], dets[:, 0]))
    return np.ascontiguousarray(dets[order])


def full_sector(M: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """Every determinant of the (n_alpha, n_beta) sector, canonical order."""
    A = [bits(c) for c in itertools.combinations(range(M), n_alpha)]
    B = [bits(c) for c in itertools.combinations(range(M), n_beta)]
    dets = np.array([(a, b) for a in A for b in B], dtype=np.uint64).reshape(-1, 2)
    return canonical_sort(dets)


def _rand_excite(rng, occ, vir, k):
    holes = rng.choice(len(occ), size=k, replace=False)
    parts = rng.choice(len(vir), size=k, replace=False)
    return [occ[i] for i in holes], [vir[a] for a in parts]


def sample_dets(M: int, n_alpha: int, n_beta: int, ref_a, ref_b, n: int, seed: int) -> np.ndarray:
    """A set of n distinct determinants grown rank by rank around the reference.

    Rank 0 (the reference), then all singles, then all doubles are added while they
    fit; the first rank that does not fit, and ranks 3-4 after it, are sampled
    uniformly at random (random hole/particle choices on each spin string).
    """
    rng = np.random.default_rng(seed)
    occ_a, occ_b = list(ref_a), list(ref_b)
    vir_a = [p for p in range(M) if p not in ref_a]
    vir_b = [p for p in range(M) if p not in ref_b]
    ra, rb = bits(ref_a), bits(ref_b)
    out = {(ra, rb)}

    def excite(s, holes, parts):
        for i in holes:
            s &= ~(1 << i)
        for a in parts:
            s |= 1 << a
        return s

    def all_rank(k):
        res = []
        for ka in range(0, k + 1):
            kb = k - ka
            if ka > min(len(occ_a), len(vir_a)) or kb > min(len(occ_b), len(vir_b)):
                continue
            for ha in itertools.combinations(occ_a, ka):
                for pa in itertools.combinations(vir_a, ka):
                    a = excite(ra, ha, pa)
                    for hb in itertools.combinations(occ_b, kb):
                        for pb in itertools.combinations(vir_b, kb):
                            res.append((a, excite(rb, hb, pb)))
        return res

    def count_rank(k):
        c = 0
        for ka in range(0, k + 1):
            kb = k - ka
            c += (math.comb(len(occ_a), ka) * math.comb(len(vir_a), ka)
                  * math.comb(len(occ_b), kb) * math.comb(len(vir_b), kb))
        return c

    k = 1
    while len(out) < n and k <= 2:
        cnt = count_rank(k)
        if cnt == 0:
            k += 1
            continue
        if len(out) + cnt <= n:
            out.update(all_rank(k))
            k += 1
        else:
            break
    # random fill from rank k (if it did not fit) and higher ranks up to 4
    ranks = [r for r in range(k, 5) if count_rank(r) > 0]
    weights = np.array([math.log(count_rank(r)) + 1.0 for r in ranks])
    weights = weights / weights.sum()
    guard = 0
    while len(out) < n and ranks:
        r = int(rng.choice(ranks, p=weights))
        splits = [(ka, r - ka) for ka in range(r + 1)
                  if ka <= min(len(occ_a), len(vir_a)) and r - ka <= min(len(occ_b), len(vir_b))]
        sw = np.array([math.comb(len(occ_a), ka) * math.comb(len(vir_a), ka)
                       * math.comb(len(occ_b), kb) * math.comb(len(vir_b), kb)
                       for ka, kb in splits], dtype=float)
        ka, kb = splits[int(rng.choice(len(splits), p=sw / sw.sum()))]
        ha, pa = _rand_excite(rng, occ_a, vir_a, ka)
        hb, pb = _rand_excite(rng, occ_b, vir_b, kb)
        out.add((excite(ra, ha, pa), excite(rb, hb, pb)))
        guard += 1
        if guard > 50 * n + 10000:
            raise RuntimeError("sector too small for the requested number of dets")
    dets = np.array(sorted(out), dtype=np.uint64).reshape(-1, 2)
    return canonical_sort(dets)


def random_dets(M: int, n_alpha: int, n_beta: int, n: int, seed: int) -> np.ndarray:
    """n distinct uniformly random determinants of the sector (canonical order)."""
    rng = np.random.default_rng(seed)
    out = set()
    while len(out) < n:
        a = bits(rng.choice(M, n_alpha, replace=False))
        b = bits(rng.choice(M, n_beta, replace=False))
        out.add((a, b))
    return canonical_sort(np.array(sorted(out), dtype=np.uint64))


# --------------------------------------------------------------------------- parameters
def param_layout(widths, n_orb: int, n_elec: int):
    """List of (name, offset, shape) for the flat parameter vector."""
    lay, off = [], 0
    L = len(widths) - 1
    for l in range(L):
        wshape = (widths[l], widths[l + 1])
        lay.append((f"W{l + 1}", off, wshape))
        off += wshape[0] * wshape[1]
        lay.append((f"b{l + 1}", off, (widths[l + 1],)))
        off += widths[l + 1]
    lay.append(("Phi0", off, (n_orb, n_elec)))
    off += n_orb * n_elec
    return lay, off


def init_theta(widths, M: int, n_alpha: int, n_beta: int, ref_a, ref_b, seed_w: int,
               seed_phi: int, out_scale: float = 1.0, bias_scale: float = 0.0) -> np.ndarray:
    """Flat float32 theta: Glorot-uniform weights (output layer times out_scale),
    biases zero (or U(-bias_scale, bias_scale) for tests), Phi0 = reference
    occupation columns (alpha columns first) + N(0, 1e-3^2)."""
    n_orb, n_elec = 2 * M, n_alpha + n_beta
    assert widths[0] == n_orb and widths[-1] == n_orb * n_elec
    lay, total = param_layout(widths, n_orb, n_elec)
    rng = np.random.default_rng(seed_w)
    theta = np.zeros(total, dtype=np.float64)
    L = len(widths) - 1
    for name, off, shape in lay:
        size = int(np.prod(shape))
        if name.startswith("W"):
            l = int(name[1:])
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            w = rng.uniform(-lim, lim, size=size)
            if l == L:
                w = w * out_scale
            theta[off:off + size] = w
        elif name.startswith("b") and bias_scale > 0:
            theta[off:off + size] = rng.uniform(-bias_scale, bias_scale, size=size)
    rng2 = np.random.default_rng(seed_phi)
    phi0 = np.zeros((n_orb, n_elec))
    occ = list(ref_a) + [M + p for p in ref_b]
    for k, p in enumerate(occ):
        phi0[p, k] = 1.0
    phi0 += rng2.normal(0.0, 1e-3, size=phi0.shape)
    off = lay[-1][1]
    theta[off:off + phi0.size] = phi0.reshape(-1)
    return theta.astype(np.float32)


def unpack_theta(theta, widths, n_orb: int, n_elec: int) -> dict:
    lay, total = param_layout(widths, n_orb, n_elec)
    assert theta.shape[0] == total
    return {name: theta[off:off + int(np.prod(shape))].reshape(shape) for name, off, shape in lay}


# --------------------------------------------------------------------------- bundles
@dataclass
class Problem:
    wl: Workload
    h: np.ndarray
    eri: np.ndarray
    e_core: float
    ref_a: list
    ref_b: list
    dets: np.ndarray
    theta: np.ndarray
    extra: dict = field(default_factory=dict)


def make_problem(wl: Workload, n_dets: int | None = None, out_scale: float = 1.0,
                 bias_scale: float = 0.0, integral_seed: int | None = None) -> Problem:
    """Integrals, S and theta for a workload; seeds 1000+, 2000+, 3000+, 4000+ index."""
    s = wl.seed
    h, eri, ec = make_integrals(wl.M, wl.rank, 1000 + s if integral_seed is None else integral_seed,
                                lattice=wl.lattice, xi=wl.xi)
    ra, rb = reference_occupation(h, wl.n_alpha, wl.n_beta)
    n = wl.n_dets if n_dets is None else n_dets
    if n == 0:
        dets = full_sector(wl.M, wl.n_alpha, wl.n_beta)
    else:
        dets = sample_dets(wl.M, wl.n_alpha, wl.n_beta, ra, rb, n, 4000 + s)
    theta = init_theta(wl.widths, wl.M, wl.n_alpha, wl.n_beta, ra, rb, 2000 + s, 3000 + s,
                       out_scale=out_scale, bias_scale=bias_scale)
    return Problem(wl, h, eri, ec, ra, rb, dets, theta)


def make_curve(wl: Workload, n_geoms: int = 64, size_lo: int = 10, size_hi: int = 16, out_scale: float = 1e-2,
               sizes=None) -> list:
    """A synthetic dissociation curve: integrals (1-t) A + t B between two seeded
    endpoint sets, t = g / (n_geoms - 1); |S_g| = round(2^(size_lo + (size_hi - size_lo) u_g))
    with u_g ~ U(0, 1) (or the given sizes); an independent theta per geometry."""
    s = wl.seed
    hA, eA, _ = make_integrals(wl.M, wl.rank, 1000 + 10 * s + 1, lattice=wl.lattice, xi=wl.xi)
    hB, eB, _ = make_integrals(wl.M, wl.rank, 1000 + 10 * s + 2, lattice=wl.lattice, xi=wl.xi)
    rng = np.random.default_rng(4000 + 10 * s)
    if sizes is None:
        sizes = [int(round(2.0 ** (size_lo + (size_hi - size_lo) * u))) for u in rng.uniform(size=n_geoms)]
    out = []
    for g in range(n_geoms):
        t = g / max(n_geoms - 1, 1)
        h, eri = interpolate_integrals(hA, eA, hB, eB, t)
        ra, rb = reference_occupation(h, wl.n_alpha, wl.n_beta)
        dets = sample_dets(wl.M, wl.n_alpha, wl.n_beta, ra, rb, int(sizes[g]), 4000 + 100 * s + g)
        theta = init_theta(wl.widths, wl.M, wl.n_alpha, wl.n_beta, ra, rb, 2000 + 100 * s + g, 3000 + 100 * s + g,
                           out_scale=out_scale)
        out.append(Problem(wl, h, eri, 0.0, ra, rb, dets, theta, {"t": t}))
    return out
