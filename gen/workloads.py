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


# ---------------------------------------------------------------------------
# four subsystems: block l, site 1, site 2, block r (the l-1-1-r strategy)
# ---------------------------------------------------------------------------


@dataclass
class Problem4:
    """One superblock written over its four subsystems (Sec. "l-1-1-r strategy"):
    ``spaces`` = [l, s1, s2, r], ``ops`` = one operator list per subsystem,
    ``terms`` int32 [nterm, 4] with ``coef`` [nterm]: term k is
    coef[k] * ops[0][a] (x) ops[1][b] (x) ops[2][c] (x) ops[3][d]."""

    spaces: List[Space]
    target: np.ndarray
    ops: List[List[Operator]]
    terms: np.ndarray
    coef: np.ndarray
    name: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.target = np.asarray(self.target, dtype=np.int32).reshape(-1)
        self.terms = np.ascontiguousarray(np.asarray(self.terms, dtype=np.int32).reshape(-1, 4))
        self.coef = np.ascontiguousarray(np.asarray(self.coef, dtype=np.float64).reshape(-1))


def spin_site():
    """One spin-1/2 site in sector form: labels 2 S^z = -1 (down), +1 (up);
    operators I, Sz, S+, S- (Eq. 3)."""
    space = Space(np.array([[-1], [1]], dtype=np.int32), np.array([1, 1]))
    ops = [Operator("identity", name="I"),
           Operator("diag", diag=np.array([-0.5, 0.5]), name="Sz"),
           Operator("dense", src=[0], dst=[1], blocks=[np.ones((1, 1))], name="S+"),
           Operator("dense", src=[1], dst=[0], blocks=[np.ones((1, 1))], name="S-")]
    return space, ops


def heisenberg_l11r(n_left: int = 4, n_right: int = 4, J: float = 1.0, delta: float = 1.0) -> Problem4:
    """Open spin-1/2 Heisenberg chain (Eq. 1-3) of n_left + 2 + n_right sites
    as exact block l, two single sites and exact block r; target S^z = 0.

    Operator lists: l and r as in :func:`heisenberg_exact` (I, H, S+, S-, Sz,
    coupling operators on the site next to the middle), sites I, Sz, S+, S-.
    Eleven terms: H_l, H_r, and the three bonds l-1, 1-2, 2-r.
    """
    L, opsL = _spin_block(n_left, n_left, J, delta)
    R, opsR = _spin_block(n_right, 1, J, delta)
    S, opsS = spin_site()
    S2, opsS2 = spin_site()
    h = 0.5 * J
    z = J * delta
    # (l, s1, s2, r): l ops I0 H1 S+2 S-3 Sz4; site ops I0 Sz1 S+2 S-3
    terms = [(1, 0, 0, 0), (0, 0, 0, 1),
             (2, 3, 0, 0), (3, 2, 0, 0), (4, 1, 0, 0),
             (0, 2, 3, 0), (0, 3, 2, 0), (0, 1, 1, 0),
             (0, 0, 2, 3), (0, 0, 3, 2), (0, 0, 1, 4)]
    coef = [1.0, 1.0, h, h, z, h, h, z, h, h, z]
    return Problem4([L, S, S2, R], [0], [opsL, opsS, opsS2, opsR], terms, coef,
                    name=f"heisenberg_l11r_{n_left}+1+1+{n_right}",
                    meta={"nsites": n_left + n_right + 2, "J": J, "delta": delta})


def hubbard_site(t: float = 1.0, U: float = 4.0):
    """One spin-1/2 Hubbard site (Eq. 4-8) in sector form, labels (N_up, N_dn):
    operators I, H = U n_up n_dn, n_up n_dn, n_up, n_dn, the parity P = (-1)^N,
    and c_sigma, c_sigma^dagger with their products with P (the single-site
    block of :func:`hubbard_exact`: modes ordered down, up)."""
    space, o = _hubbard_block(1, 1, t, U)
    nn = Operator("diag", diag=_sector_values(space, space.labels[:, 0] * space.labels[:, 1]), name="nn")
    nu = Operator("diag", diag=_sector_values(space, space.labels[:, 0]), name="nu")
    nd = Operator("diag", diag=_sector_values(space, space.labels[:, 1]), name="nd")
    par = Operator("diag", diag=_sector_values(space, (-1.0) ** (space.labels[:, 0] + space.labels[:, 1])),
                   name="P")
    names = ["cdag_up", "c_up", "cdag_dn", "c_dn", "cdagP_up", "Pc_up", "cdagP_dn", "Pc_dn"]
    ops = [o["I"], o["H"], nn, nu, nd, par] + [o[k] for k in names]
    return space, ops


def _hubbard_l11r_terms(t: float, with_site_u: bool, U: float):
    """Terms over (l, s1, s2, r) for a Hubbard chain; site op indices as in
    :func:`hubbard_site` (I0 H1 nn2 nu3 nd4 P5 cdag_up6 c_up7 cdag_dn8 c_dn9
    cdagP_up10 Pc_up11 cdagP_dn12 Pc_dn13); block op order
    I0 H1 cdagP_up2 Pc_up3 cdagP_dn4 Pc_dn5 (left) and I0 H1 c_up2 cdag_up3
    c_dn4 cdag_dn5 (right).  Hopping across a cut: the creation operator of the
    earlier subsystem times its parity, then the annihilator of the later
    one, and the Hermitian conjugate (Jordan-Wigner, Eq. 5-8)."""
    terms = [(1, 0, 0, 0), (0, 0, 0, 1)]
    coef = [1.0, 1.0]
    if with_site_u:
        terms += [(0, 1, 0, 0), (0, 0, 1, 0)]  # U n_up n_dn on each site
        coef += [1.0, 1.0]
    # l - s1: cdagP_l c_1 and P c_l cdag_1 per spin
    terms += [(2, 7, 0, 0), (3, 6, 0, 0), (4, 9, 0, 0), (5, 8, 0, 0)]
    # s1 - s2
    terms += [(0, 10, 7, 0), (0, 11, 6, 0), (0, 12, 9, 0), (0, 13, 8, 0)]
    # s2 - r
    terms += [(0, 0, 10, 2), (0, 0, 11, 3), (0, 0, 12, 4), (0, 0, 13, 5)]
    coef += [-t] * 12
    return terms, coef


def hubbard_l11r_exact(n_left: int = 1, n_right: int = 1, t: float = 1.0, U: float = 4.0) -> Problem4:
    """Spin-1/2 Hubbard chain of n_left + 2 + n_right sites (Eq. 4-8) as exact
    block l, two sites and exact block r, at half filling."""
    L, oL = _hubbard_block(n_left, n_left, t, U)
    R, oR = _hubbard_block(n_right, 1, t, U)
    S, opsS = hubbard_site(t, U)
    S2, opsS2 = hubbard_site(t, U)
    opsL = [oL[k] for k in ["I", "H", "cdagP_up", "Pc_up", "cdagP_dn", "Pc_dn"]]
    opsR = [oR[k] for k in ["I", "H", "c_up", "cdag_up", "c_dn", "cdag_dn"]]
    terms, coef = _hubbard_l11r_terms(t, True, U)
    N = n_left + n_right + 2
    return Problem4([L, S, S2, R], [N // 2, N // 2], [opsL, opsS, opsS2, opsR], terms, coef,
                    name=f"hubbard_l11r_{n_left}+1+1+{n_right}", meta={"nsites": N, "t": t, "U": U})


def hubbard_l11r_synthetic(m: int = 512, seed: int = 8642, t: float = 1.0, U: float = 4.0) -> Problem4:
    """Hubbard superblock of four subsystems: random blocks l and r of m states
    with the Gaussian (N_up, N_dn) sectors of :func:`hubbard_space` (H block,
    cdag maps with the block parity, as in :func:`hubbard_synthetic`; l from
    ``seed``, r from ``seed + 1``) and two exact Hubbard sites (U n_up n_dn).
    Sixteen terms: H_l, H_r, U on each site, four hoppings across each of the
    three cuts.  Target: the block reference fillings plus one particle of
    each spin on the two sites (labels measured from the blocks' reference)."""
    space = hubbard_space(m)
    opsL_all = _hub_side(space, m, seed, True)
    opsR_all = _hub_side(space, m, seed + 1, False)
    opsL = [opsL_all[k] for k in (0, 1, 5, 6, 7, 8)]
    opsR = [opsR_all[k] for k in (0, 1, 5, 6, 7, 8)]
    S, opsS = hubbard_site(t, U)
    S2, opsS2 = hubbard_site(t, U)
    terms, coef = _hubbard_l11r_terms(t, True, U)
    return Problem4([space, S, S2, Space(space.labels, space.dims)], [1, 1], [opsL, opsS, opsS2, opsR],
                    terms, coef, name=f"hubbard_l11r_m{m}", seed=seed, meta={"m": m, "t": t, "U": U})


def random_problem4(seed: int, rank: int = 1, nsec: int = 4, dmax: int = 7, site_dmax: int = 2,
                    nops: int = 3, nterm: int = 6, p_zero: float = 0.15, p_drop: float = 0.2) -> Problem4:
    """Random four-subsystem structure: ragged block spaces (zero and unit
    dimensions), small site spaces with sectors of dimension up to site_dmax,
    every operator kind, missing blocks; every term conserves the target."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if rank == 1:
        pool = [(a,) for a in range(-3, 4)]
    else:
        pool = [(a, b) for a in range(-2, 3) for b in range(-2, 3)]
    unit = [np.zeros(rank, dtype=np.int32)]
    for a in range(rank):
        e = np.zeros(rank, dtype=np.int32)
        e[a] = 1
        unit += [e, -e]

    def make_space(k, dmax_):
        k = min(k, len(pool))
        pick = sorted(rng.choice(len(pool), size=k, replace=False))
        labels = np.array([pool[i] for i in pick], dtype=np.int32)
        dims = rng.integers(1, dmax_ + 1, size=k)
        dims[rng.random(k) < p_zero] = 0
        return Space(labels, dims)

    spaces = [make_space(nsec, dmax), make_space(3, site_dmax), make_space(3, site_dmax), make_space(nsec, dmax)]
    for sp in spaces[1:3]:  # sites keep every sector non-empty
        sp.dims[sp.dims == 0] = 1

    def make_op(space, sh):
        if sh is None:
            return Operator("diag", diag=rng.standard_normal(space.m), name="D")
        src, dst, blocks = [], [], []
        for s in range(space.nsec):
            d = space.index(space.labels[s] + sh)
            if d < 0 or rng.random() < p_drop:
                continue
            src.append(s)
            dst.append(d)
            blocks.append(rng.standard_normal((int(space.dims[d]), int(space.dims[s]))))
        return Operator("dense", src=src, dst=dst, blocks=blocks, name="M")

    # operator j of every subsystem has shift shifts[j]; shift None = diagonal
    shifts = [[None] + [unit[int(rng.integers(len(unit)))] for _ in range(nops - 1)] for _ in range(4)]
    ops = [[Operator("identity", name="I")] + [make_op(spaces[s], sh) for sh in shifts[s]] for s in range(4)]

    def shift(s, j):
        if j == 0 or shifts[s][j - 1] is None:
            return np.zeros(rank, dtype=np.int32)
        return shifts[s][j - 1]

    terms = []
    while len(terms) < nterm:
        pick = [int(rng.integers(len(ops[s]))) for s in range(3)]
        tot = sum(shift(s, pick[s]) for s in range(3))
        ok = [d for d in range(len(ops[3])) if np.array_equal(shift(3, d), -tot)]
        if not ok:
            continue
        terms.append(tuple(pick) + (ok[int(rng.integers(len(ok)))],))
    # a target reachable by some non-empty quadruple
    cand = [(i, j, k, l) for i in range(spaces[0].nsec) for j in range(spaces[1].nsec)
            for k in range(spaces[2].nsec) for l in range(spaces[3].nsec)
            if spaces[0].dims[i] and spaces[1].dims[j] and spaces[2].dims[k] and spaces[3].dims[l]]
    q = cand[int(rng.integers(len(cand)))]
    target = sum(spaces[s].labels[q[s]] for s in range(4))
    coef = rng.standard_normal(len(terms))
    return Problem4(spaces, target, ops, terms, coef, name=f"random4_{seed}_r{rank}", seed=seed)
