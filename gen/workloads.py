"""Workload recipes: exact small chains and seeded synthetic superblocks.

Every array produced here is an *input*.  Nothing in this module evaluates a
projection, a Davidson step or an eigenvalue; it only builds sector tables and
operator blocks the way the paper's models (Eq. 1-8) and the synthetic
workloads need them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# containers
# ---------------------------------------------------------------------------


@dataclass
class Space:
    """Sector table of one (enlarged) block.

    ``labels``: int32 ``[nsec, rank]``, strictly ascending lexicographically.
    ``dims``: int64 ``[nsec]`` (>= 0).
    """

    labels: np.ndarray
    dims: np.ndarray

    def __post_init__(self):
        self.labels = np.ascontiguousarray(np.asarray(self.labels, dtype=np.int32))
        if self.labels.ndim == 1:
            self.labels = self.labels[:, None].copy()
        self.dims = np.ascontiguousarray(np.asarray(self.dims, dtype=np.int64))

    @property
    def nsec(self) -> int:
        return int(self.dims.shape[0])

    @property
    def rank(self) -> int:
        return int(self.labels.shape[1])

    @property
    def m(self) -> int:
        return int(self.dims.sum())

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.nsec + 1, dtype=np.int64)
        np.cumsum(self.dims, out=off[1:])
        return off

    def index(self, label) -> int:
        """Sector index of ``label`` or -1."""
        lab = np.asarray(label, dtype=np.int32).reshape(-1)
        hit = np.nonzero((self.labels == lab).all(axis=1))[0]
        return int(hit[0]) if hit.size else -1


@dataclass
class Operator:
    """Block-sparse operator on a space (kind ``identity``, ``diag`` or ``dense``)."""

    kind: str
    src: Optional[np.ndarray] = None
    dst: Optional[np.ndarray] = None
    blocks: Optional[List[np.ndarray]] = None
    diag: Optional[np.ndarray] = None
    name: str = ""

    def __post_init__(self):
        if self.kind == "dense":
            self.src = np.asarray(self.src, dtype=np.int32)
            self.dst = np.asarray(self.dst, dtype=np.int32)
            self.blocks = [np.ascontiguousarray(b, dtype=np.float64) for b in self.blocks]
        elif self.kind == "diag":
            self.diag = np.ascontiguousarray(self.diag, dtype=np.float64)
        elif self.kind != "identity":
            raise ValueError(f"unknown operator kind {self.kind!r}")

    @property
    def nblk(self) -> int:
        return len(self.blocks) if self.kind == "dense" else 0


@dataclass
class Problem:
    """One superblock: two spaces, operator lists, terms, coefficients, target."""

    left: Space
    right: Space
    target: np.ndarray
    ops_left: List[Operator]
    ops_right: List[Operator]
    terms: np.ndarray  # int32 [nterm, 2]: (left op index, right op index)
    coef: np.ndarray  # float64 [nterm]
    name: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.target = np.asarray(self.target, dtype=np.int32).reshape(-1)
        self.terms = np.ascontiguousarray(np.asarray(self.terms, dtype=np.int32).reshape(-1, 2))
        self.coef = np.ascontiguousarray(np.asarray(self.coef, dtype=np.float64).reshape(-1))


# ---------------------------------------------------------------------------
# sector sizes
# ---------------------------------------------------------------------------


def largest_remainder(weights: Sequence[float], total: int, tie_keys: Sequence) -> np.ndarray:
    """Integer sizes proportional to ``weights`` that sum to ``total``.

    Hamilton's largest-remainder rule: floor the exact quotas, then hand the
    remaining units to the largest fractional parts.  Equal fractional parts
    are ordered by ``tie_keys`` (smaller key first).
    """
    w = np.asarray(weights, dtype=np.float64)
    quota = total * w / w.sum()
    base = np.floor(quota).astype(np.int64)
    frac = quota - base
    left = int(total - base.sum())
    order = sorted(range(len(w)), key=lambda i: (-frac[i], tie_keys[i]))
    for i in order[:left]:
        base[i] += 1
    return base


def _compact(labels: np.ndarray, dims: np.ndarray) -> Space:
    keep = dims > 0
    return Space(labels[keep], dims[keep])


def heisenberg_space(m: int, qmax: int = 10) -> Space:
    """Sector sizes proportional to binomial(2 qmax, qmax + q), q = -qmax..qmax."""
    qs = np.arange(-qmax, qmax + 1)
    w = [comb(2 * qmax, qmax + int(q)) for q in qs]
    dims = largest_remainder(w, m, [(abs(int(q)), int(q)) for q in qs])
    return _compact(qs[:, None], dims)


def hubbard_space(m: int, half_width: int = 9, sigma: float = 3.0) -> Space:
    """(N_up - N_up0, N_dn - N_dn0) sectors with a 2-D Gaussian size profile."""
    r = np.arange(-half_width, half_width + 1)
    lab = np.array([(a, b) for a in r for b in r], dtype=np.int32)
    w = np.exp(-(lab[:, 0].astype(float) ** 2 + lab[:, 1].astype(float) ** 2) / (2 * sigma * sigma))
    keys = [(int(a * a + b * b), int(a), int(b)) for a, b in lab]
    dims = largest_remainder(w, m, keys)
    return _compact(lab, dims)


# ---------------------------------------------------------------------------
# helpers for dense -> sector form (exact chains)
# ---------------------------------------------------------------------------


def _sector_form(labels_per_state: np.ndarray):
    """Group basis states by label; return (Space, permutation, sector lists)."""
    lab = np.asarray(labels_per_state, dtype=np.int32)
    if lab.ndim == 1:
        lab = lab[:, None]
    uniq = np.unique(lab, axis=0)  # lexicographically ascending
    members = []
    for u in uniq:
        members.append(np.nonzero((lab == u).all(axis=1))[0])
    dims = np.array([len(x) for x in members], dtype=np.int64)
    return Space(uniq, dims), members


def _dense_to_op(M: np.ndarray, members, name: str, want_diag: bool = False) -> Operator:
    if want_diag:
        if np.count_nonzero(M - np.diag(np.diag(M))):
            raise ValueError(f"{name} is not diagonal")
        perm = np.concatenate(members)
        return Operator("diag", diag=np.diag(M)[perm].copy(), name=name)
    src, dst, blocks = [], [], []
    for j, mj in enumerate(members):  # source sector
        for i, mi in enumerate(members):  # destination sector
            blk = M[np.ix_(mi, mj)]
            if np.count_nonzero(blk):
                src.append(j)
                dst.append(i)
                blocks.append(blk.copy())
    return Operator("dense", src=src, dst=dst, blocks=blocks, name=name)


def _embed(op2: np.ndarray, site: int, nsites: int, d: int = 2) -> np.ndarray:
    """Eq. 2: identity on every site but ``site`` (1-based)."""
    out = np.ones((1, 1))
    for j in range(1, nsites + 1):
        out = np.kron(out, op2 if j == site else np.eye(d))
    return out


# Eq. 3 (basis index 0 is spin up, S^z = +1/2)
_SP = np.array([[0.0, 1.0], [0.0, 0.0]])
_SM = np.array([[0.0, 0.0], [1.0, 0.0]])
_SZ = 0.5 * np.array([[1.0, 0.0], [0.0, -1.0]])


def _spin_block(nsites: int, edge: int, J: float, delta: float):
    """Exact enlarged block of ``nsites`` spins; edge operators on site ``edge``."""
    dim = 2 ** nsites
    H = np.zeros((dim, dim))
    for j in range(1, nsites):
        H += J * 0.5 * (_embed(_SP, j, nsites) @ _embed(_SM, j + 1, nsites)
                        + _embed(_SM, j, nsites) @ _embed(_SP, j + 1, nsites))
        H += J * delta * (_embed(_SZ, j, nsites) @ _embed(_SZ, j + 1, nsites))
    # label = 2 S^z_total = (#up - #down); site 1 is the most significant bit
    states = np.arange(dim)
    ups = np.zeros(dim, dtype=np.int64)
    for j in range(1, nsites + 1):
        bit = (states >> (nsites - j)) & 1
        ups += (bit == 0)
    labels = 2 * ups - nsites
    space, members = _sector_form(labels)
    ops = [
        Operator("identity", name="I"),
        _dense_to_op(H, members, "H"),
        _dense_to_op(_embed(_SP, edge, nsites), members, "S+"),
        _dense_to_op(_embed(_SM, edge, nsites), members, "S-"),
        _dense_to_op(_embed(_SZ, edge, nsites), members, "Sz", want_diag=True),
    ]
    return space, ops


def heisenberg_exact(n_left: int = 5, n_right: int = 5, J: float = 1.0, delta: float = 1.0,
                     seed: int = 0) -> Problem:
    """Open spin-1/2 Heisenberg chain (Eq. 1-3) split into two exact enlarged blocks.

    Labels are 2 S^z (integers); the target is S^z_total = 0.  The left block's
    coupling operators sit on its last site and the right block's on its first.
    Operator order on both sides: I, H, S+, S-, Sz.
    """
    L, opsL = _spin_block(n_left, n_left, J, delta)
    R, opsR = _spin_block(n_right, 1, J, delta)
    terms = [(1, 0), (0, 1), (2, 3), (3, 2), (4, 4)]
    coef = [1.0, 1.0, 0.5 * J, 0.5 * J, J * delta]
    return Problem(L, R, [0], opsL, opsR, terms, coef,
                   name=f"heisenberg_exact_{n_left}+{n_right}", seed=seed,
                   meta={"nsites": n_left + n_right, "J": J, "delta": delta})


# Eq. 7-8: phase factor and single-mode creation/annihilation; [1;0] empty
_PHI = np.array([[1.0, 0.0], [0.0, -1.0]])
_CDAG = np.array([[0.0, 0.0], [1.0, 0.0]])
_C = np.array([[0.0, 1.0], [0.0, 0.0]])


def _mode_op(op2: np.ndarray, mode: int, nmodes: int) -> np.ndarray:
    """Eq. 5-6: phase string on every earlier mode, identity on later ones."""
    out = np.ones((1, 1))
    for k in range(nmodes):
        out = np.kron(out, _PHI if k < mode else (op2 if k == mode else np.eye(2)))
    return out


def _hubbard_block(nsites: int, edge: int, t: float, U: float):
    """Exact spin-1/2 Hubbard block; modes ordered (site, sigma) with sigma = down, up."""
    nm = 2 * nsites
    dim = 2 ** nm
    cd = {}
    cc = {}
    for j in range(1, nsites + 1):
        for s in (0, 1):  # 0: down (sigma=-1/2), 1: up (sigma=+1/2)
            k = 2 * (j - 1) + s
            cd[(j, s)] = _mode_op(_CDAG, k, nm)
            cc[(j, s)] = _mode_op(_C, k, nm)
    H = np.zeros((dim, dim))
    for j in range(1, nsites):
        for s in (0, 1):
            hop = cd[(j, s)] @ cc[(j + 1, s)]
            H += -t * (hop + hop.T)
    for j in range(1, nsites + 1):
        H += U * (cd[(j, 1)] @ cc[(j, 1)]) @ (cd[(j, 0)] @ cc[(j, 0)])
    states = np.arange(dim)
    n_up = np.zeros(dim, dtype=np.int64)
    n_dn = np.zeros(dim, dtype=np.int64)
    for k in range(nm):
        occ = (states >> (nm - 1 - k)) & 1
        if k % 2 == 1:
            n_up += occ
        else:
            n_dn += occ
    labels = np.stack([n_up, n_dn], axis=1)
    space, members = _sector_form(labels)
    parity = np.diag((-1.0) ** (n_up + n_dn))
    ops = {"I": Operator("identity", name="I"), "H": _dense_to_op(H, members, "H")}
    for s, tag in ((1, "up"), (0, "dn")):
        cdag = cd[(edge, s)]
        c = cc[(edge, s)]
        ops[f"cdag_{tag}"] = _dense_to_op(cdag, members, f"cdag_{tag}")
        ops[f"c_{tag}"] = _dense_to_op(c, members, f"c_{tag}")
        ops[f"cdagP_{tag}"] = _dense_to_op(cdag @ parity, members, f"cdagP_{tag}")
        ops[f"Pc_{tag}"] = _dense_to_op(parity @ c, members, f"Pc_{tag}")
    return space, ops


def hubbard_exact(n_left: int = 2, n_right: int = 2, t: float = 1.0, U: float = 4.0,
                  n_up: Optional[int] = None, n_dn: Optional[int] = None) -> Problem:
    """Spin-1/2 Hubbard chain (Eq. 4-8) as two exact enlarged blocks.

    Cross-cut hopping terms take the left operator times the left parity
    (-1)^{N_L} of the source sector, which is what the Jordan-Wigner string of
    the right site's operator reduces to on the left block (Eq. 5).
    Labels are (N_up, N_dn); the default target is half filling.
    """
    N = n_left + n_right
    n_up = N // 2 if n_up is None else n_up
    n_dn = N // 2 if n_dn is None else n_dn
    L, oL = _hubbard_block(n_left, n_left, t, U)
    R, oR = _hubbard_block(n_right, 1, t, U)
    namesL = ["I", "H", "cdagP_up", "Pc_up", "cdagP_dn", "Pc_dn"]
    namesR = ["I", "H", "c_up", "cdag_up", "c_dn", "cdag_dn"]
    opsL = [oL[k] for k in namesL]
    opsR = [oR[k] for k in namesR]
    terms = [(1, 0), (0, 1), (2, 2), (3, 3), (4, 4), (5, 5)]
    coef = [1.0, 1.0, -t, -t, -t, -t]
    return Problem(L, R, [n_up, n_dn], opsL, opsR, terms, coef,
                   name=f"hubbard_exact_{n_left}+{n_right}",
                   meta={"nsites": N, "t": t, "U": U})


# ---------------------------------------------------------------------------
# synthetic superblocks
# ---------------------------------------------------------------------------


def _sym_blocks(rng, space: Space, m: int, spread: float):
    """Per-sector symmetric blocks N(0,1)/sqrt(m) plus a uniform[-spread, 0] diagonal."""
    blocks = []
    for d in space.dims:
        g = rng.standard_normal((int(d), int(d))) / np.sqrt(m)
        blocks.append(np.triu(g) + np.triu(g, 1).T)
    for b in blocks:
        b[np.diag_indices_from(b)] += rng.uniform(-spread, 0.0, b.shape[0])
    idx = np.arange(space.nsec, dtype=np.int32)
    return Operator("dense", src=idx, dst=idx, blocks=blocks, name="H")


def _shift_map(rng, space: Space, m: int, shift, name: str):
    """Dense random map sector q -> q + shift, blocks N(0,1)/sqrt(m)."""
    shift = np.asarray(shift, dtype=np.int32).reshape(-1)
    src, dst, blocks = [], [], []
    for s in range(space.nsec):
        d = space.index(space.labels[s] + shift)
        if d < 0:
            continue
        src.append(s)
        dst.append(d)
        blocks.append(rng.standard_normal((int(space.dims[d]), int(space.dims[s]))) / np.sqrt(m))
    return Operator("dense", src=src, dst=dst, blocks=blocks, name=name)


def _transpose_op(op: Operator, name: str, scale_dst=None) -> Operator:
    """Transpose of a dense operator; optional per-sector factor on the new destination."""
    blocks = []
    for k in range(op.nblk):
        bt = op.blocks[k].T.copy()
        if scale_dst is not None:
            bt *= scale_dst[int(op.src[k])]
        blocks.append(bt)
    return Operator("dense", src=op.dst.copy(), dst=op.src.copy(), blocks=blocks, name=name)


def _scaled_src(op: Operator, factor, name: str) -> Operator:
    blocks = [op.blocks[k] * factor[int(op.src[k])] for k in range(op.nblk)]
    return Operator("dense", src=op.src.copy(), dst=op.dst.copy(), blocks=blocks, name=name)


def _sector_values(space: Space, values) -> np.ndarray:
    return np.repeat(np.asarray(values, dtype=np.float64), space.dims)


def _heis_side(space: Space, m: int, seed: int, j2: bool):
    rng = np.random.Generator(np.random.PCG64(seed))
    H = _sym_blocks(rng, space, m, 50.0)
    Sp = _shift_map(rng, space, m, [1], "S+")
    ops = [Operator("identity", name="I"), H,
           Operator("diag", diag=_sector_values(space, space.labels[:, 0]), name="Sz"),
           Sp, _transpose_op(Sp, "S-")]
    if j2:
        Spp = _shift_map(rng, space, m, [1], "S'+")
        ops += [Spp, _transpose_op(Spp, "S'-"),
                Operator("diag", diag=rng.uniform(-0.5, 0.5, m), name="S'z")]
    return ops


def heisenberg_synthetic(m: int = 1024, seed: int = 1234, J: float = 1.0, delta: float = 1.0,
                         qmax: int = 10) -> Problem:
    """Two-site Heisenberg superblock with random blocks (five terms, target S^z = 0).

    Operator order on each side: I, H, Sz, S+, S- (S- is the transpose of S+).
    Left draws from ``seed``, right from ``seed + 1``.
    """
    space = heisenberg_space(m, qmax)
    opsL = _heis_side(space, m, seed, False)
    opsR = _heis_side(space, m, seed + 1, False)
    terms = [(1, 0), (0, 1), (3, 4), (4, 3), (2, 2)]
    coef = [1.0, 1.0, 0.5 * J, 0.5 * J, J * delta]
    return Problem(space, Space(space.labels, space.dims), [0], opsL, opsR, terms, coef,
                   name=f"heisenberg_m{m}", seed=seed, meta={"m": m})


def j1j2_synthetic(m: int = 1024, seed: int = 1234, J1: float = 1.0, J2: float = 0.5) -> Problem:
    """Heisenberg superblock plus next-nearest S.S terms (eight terms).

    ``meta['coef_basis']`` is the ``[nterm, 3]`` matrix with
    coef = basis @ (1, J1, J2), so derivatives with respect to J1 and J2 are
    its second and third columns.
    """
    space = heisenberg_space(m)
    opsL = _heis_side(space, m, seed, True)
    opsR = _heis_side(space, m, seed + 1, False)
    terms = [(1, 0), (0, 1), (3, 4), (4, 3), (2, 2), (5, 4), (6, 3), (7, 2)]
    basis = np.array([[1, 0, 0], [1, 0, 0], [0, 0.5, 0], [0, 0.5, 0], [0, 1, 0],
                      [0, 0, 0.5], [0, 0, 0.5], [0, 0, 1]], dtype=np.float64)
    coef = basis @ np.array([1.0, J1, J2])
    return Problem(space, Space(space.labels, space.dims), [0], opsL, opsR, terms, coef,
                   name=f"j1j2_m{m}", seed=seed,
                   meta={"m": m, "J1": J1, "J2": J2, "coef_basis": basis})


def _hub_side(space: Space, m: int, seed: int, left: bool):
    rng = np.random.Generator(np.random.PCG64(seed))
    H = _sym_blocks(rng, space, m, 50.0)
    nn = Operator("diag", diag=rng.uniform(0.0, 1.0, m), name="nn")
    nu = Operator("diag", diag=rng.uniform(0.0, 1.0, m), name="nu")
    nd = Operator("diag", diag=rng.uniform(0.0, 1.0, m), name="nd")
    cup = _shift_map(rng, space, m, [1, 0], "cdag_up")
    cdn = _shift_map(rng, space, m, [0, 1], "cdag_dn")
    ops = [Operator("identity", name="I"), H, nn, nu, nd]
    if left:
        # parity (-1)^{N} of a sector; the reference filling is even
        par = (-1.0) ** (space.labels[:, 0] + space.labels[:, 1])
        ops += [_scaled_src(cup, par, "cdagP_up"), _transpose_op(cup, "Pc_up", par),
                _scaled_src(cdn, par, "cdagP_dn"), _transpose_op(cdn, "Pc_dn", par)]
    else:
        ops += [_transpose_op(cup, "c_up"), cup, _transpose_op(cdn, "c_dn"), cdn]
    return ops


def hubbard_synthetic(m: int = 2048, seed: int = 4321, t: float = 1.0, U: float = 4.0) -> Problem:
    """Two-site Hubbard superblock with U(1)xU(1) sectors and twelve terms.

    Operator order, left: I, H, nn, nu, nd, cdag_up P, P c_up, cdag_dn P, P c_dn;
    right: I, H, nn, nu, nd, c_up, cdag_up, c_dn, cdag_dn.  The interaction is
    written particle-hole symmetrically, U(n_up n_dn) - U/2 (n_up + n_dn), per
    side; the hopping crosses the cut with the fermionic parity on the left.
    """
    space = hubbard_space(m)
    opsL = _hub_side(space, m, seed, True)
    opsR = _hub_side(space, m, seed + 1, False)
    terms = [(1, 0), (0, 1), (2, 0), (0, 2), (3, 0), (0, 3), (4, 0), (0, 4),
             (5, 5), (6, 6), (7, 7), (8, 8)]
    coef = [1.0, 1.0, U, U, -U / 2, -U / 2, -U / 2, -U / 2, -t, -t, -t, -t]
    return Problem(space, Space(space.labels, space.dims), [0, 0], opsL, opsR, terms, coef,
                   name=f"hubbard_m{m}", seed=seed, meta={"m": m, "t": t, "U": U})


BATCH_SIZES = (256, 512, 768, 1024, 1536, 2048)


def batched_heisenberg(count: int = 64, seed: int = 777) -> List[Problem]:
    """``count`` independent Heisenberg superblocks with m drawn from BATCH_SIZES."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ms = rng.choice(np.array(BATCH_SIZES), size=count)
    return [heisenberg_synthetic(int(m), seed=seed + 10 * (i + 1)) for i, m in enumerate(ms)]


# ---------------------------------------------------------------------------
# random structures for edge-case testing
# ---------------------------------------------------------------------------


def random_problem(seed: int, rank: int = 1, nsec: int = 5, dmax: int = 12,
                   nops: int = 4, nterm: int = 6, p_zero: float = 0.15,
                   p_drop: float = 0.2, square: bool = False) -> Problem:
    """Random sector structure with every operator kind and ragged block sizes.

    Sectors may have dimension 0 or 1, left and right spaces differ, dense
    operators shift labels by 0 or a unit vector and may miss blocks.  Every
    term conserves the target label.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if rank == 1:
        pool = [(a,) for a in range(-4, 5)]
    else:
        pool = [(a, b) for a in range(-2, 3) for b in range(-2, 3)]

    def make_space():
        k = min(nsec, len(pool))
        pick = sorted(rng.choice(len(pool), size=k, replace=False))
        labels = np.array([pool[i] for i in pick], dtype=np.int32)
        dims = rng.integers(1, dmax + 1, size=k)
        dims[rng.random(k) < p_zero] = 0
        return Space(labels, dims)

    L = make_space()
    R = L if square else make_space()
    # choose a target reachable by at least one non-empty pair
    cand = [(i, j) for i in range(L.nsec) for j in range(R.nsec) if L.dims[i] and R.dims[j]]
    i, j = cand[int(rng.integers(len(cand)))]
    target = L.labels[i] + R.labels[j]

    unit = [np.zeros(rank, dtype=np.int32)]
    for a in range(rank):
        e = np.zeros(rank, dtype=np.int32)
        e[a] = 1
        unit += [e, -e]

    def make_ops(space, shifts):
        ops = [Operator("identity", name="I")]
        for sh in shifts:
            if sh is None:
                ops.append(Operator("diag", diag=rng.standard_normal(space.m), name="D"))
                continue
            src, dst, blocks = [], [], []
            for s in range(space.nsec):
                d = space.index(space.labels[s] + sh)
                if d < 0 or rng.random() < p_drop:
                    continue
                src.append(s)
                dst.append(d)
                blocks.append(rng.standard_normal((int(space.dims[d]), int(space.dims[s]))))
            ops.append(Operator("dense", src=src, dst=dst, blocks=blocks, name="M"))
        return ops

    shiftsL = [None] + [unit[int(rng.integers(len(unit)))] for _ in range(nops - 1)]
    opsL = make_ops(L, shiftsL)
    # right operators: for every left shift, one with the opposite shift
    shiftsR = [None] + [(-s if s is not None else None) for s in shiftsL[1:]]
    opsR = make_ops(R, shiftsR)

    def shift_of(ops, shifts, k):
        if k == 0 or shifts[k - 1] is None:
            return np.zeros(rank, dtype=np.int32)
        return shifts[k - 1]

    terms = []
    for _ in range(nterm):
        a = int(rng.integers(len(opsL)))
        sa = shift_of(opsL, shiftsL, a)
        ok = [b for b in range(len(opsR)) if np.array_equal(shift_of(opsR, shiftsR, b), -sa)]
        b = ok[int(rng.integers(len(ok)))]
        terms.append((a, b))
    coef = rng.standard_normal(len(terms))
    return Problem(L, R, target, opsL, opsR, terms, coef, name=f"random_{seed}_r{rank}", seed=seed)


def start_vector(n: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) start vector of length n (PCG64); the caller normalizes."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


CONFIG_NAMES = {
    1: "heisenberg_exact_10site",
    2: "heisenberg_m1024",
    3: "hubbard_m2048",
    4: "batched_heisenberg_64",
    5: "j1j2_m1024",
}


def config(i: int, seed: Optional[int] = None):
    """The five workloads: exact 10-site chain, Heisenberg m=1024, Hubbard
    m=2048, 64 batched Heisenberg members, J1-J2 m=1024."""
    if i == 1:
        return heisenberg_exact(5, 5)
    if i == 2:
        return heisenberg_synthetic(1024, seed=1234 if seed is None else seed)
    if i == 3:
        return hubbard_synthetic(2048, seed=4321 if seed is None else seed)
    if i == 4:
        return batched_heisenberg(64, seed=777 if seed is None else seed)
    if i == 5:
        return j1j2_synthetic(1024, seed=2468 if seed is None else seed)
    raise ValueError(i)
