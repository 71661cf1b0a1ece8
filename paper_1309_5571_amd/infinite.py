"""Infinite-lattice DMRG (Alg. 1) and finite-lattice sweeps for the open
spin-1/2 XXZ (Heisenberg) chain, every numerical step on the device through
the C ABI.

One iteration: enlarge the block by one site (dmrg_place_blocks), form the
superblock of two mirror-image enlarged blocks in the S^z = 0 sector, find its
lowest eigenstate (dmrg_davidson), build the left block's density matrix
(dmrg_density), diagonalize it sector by sector (dmrg_eigh_blocks), keep the m
states of largest weight (dmrg_truncate) and take the block's operators to
the kept basis (dmrg_renormalize).  The chain grows by two sites per
iteration (Sec. "The DMRG algorithm").  `run_finite` continues at fixed size
with sweeps of the centre, renormalizing the right block from the right-side
density matrix on the way back.

Blocks carry four operators in dense sector form: the block Hamiltonian H and
the spin operators S+, S-, Sz of the site at the block's inner edge.  Labels
are 2 S^z.  The right block is the mirror image of the left one, so the same
operator data serves both sides.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from . import _native as N

OPS = ("H", "Sp", "Sm", "Sz")


@dataclass
class DevOp:
    """Dense sector-form operator whose blocks live in one device tensor."""
    src: np.ndarray  # int32 [nblk] source sector
    dst: np.ndarray  # int32 [nblk] destination sector
    off: np.ndarray  # int64 [nblk] element offset of each row-major block
    device_data: object  # torch float64 tensor
    kind: str = "dense"


@dataclass
class Block:
    labels: np.ndarray  # int32 [nsec], ascending
    dims: np.ndarray  # int64 [nsec]
    ops: Dict[str, DevOp]
    nsites: int


@dataclass
class _Space:
    labels: np.ndarray
    dims: np.ndarray


@dataclass
class _Identity:
    kind: str = "identity"


@dataclass
class _Superblock:
    left: _Space
    right: _Space
    target: np.ndarray
    ops_left: list
    ops_right: list
    terms: np.ndarray
    coef: np.ndarray


@dataclass
class StepResult:
    nsites: int  # sites of the superblock
    energy: float
    discarded: float
    kept: int
    iterations: int
    retries: int = 0  # Davidson runs restarted from a new random vector after a breakdown


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(dev):
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def site_block(device) -> Block:
    """One spin: sectors 2S^z = -1 (down), +1 (up)."""
    import torch

    def op(src, dst, vals):
        t = torch.tensor(vals, dtype=torch.float64, device=device)
        return DevOp(np.array(src, np.int32), np.array(dst, np.int32), np.arange(len(vals), dtype=np.int64), t)

    return Block(np.array([-1, 1], np.int32), np.array([1, 1], np.int64),
                 {"H": op([0, 1], [0, 1], [0.0, 0.0]), "Sp": op([0], [1], [1.0]), "Sm": op([1], [0], [1.0]),
                  "Sz": op([0, 1], [0, 1], [-0.5, 0.5])}, 1)


# site operators as (source site state, destination site state, value); state 0 = down, 1 = up
_SITE = {"I": [(0, 0, 1.0), (1, 1, 1.0)], "Sp": [(0, 1, 1.0)], "Sm": [(1, 0, 1.0)], "Sz": [(0, 0, -0.5), (1, 1, 0.5)]}
_SIGMA = (-1, 1)


def enlarge(B: Block, J: float = 1.0, delta: float = 1.0) -> Block:
    """Block + one site (Alg. 1, step 2), in sector form:
    H' = H (x) I + J/2 (S+ (x) S- + S- (x) S+) + J delta Sz (x) Sz, and the new
    edge operators I (x) S+, I (x) S-, I (x) Sz.  Enlarged sector mu holds the
    parts (lambda, sigma) with lambda + sigma = mu, spin down first."""
    import torch

    dev = B.ops["H"].device_data.device
    lab = {int(l): i for i, l in enumerate(B.labels)}
    mus = sorted({int(l) + s for l in B.labels for s in _SIGMA})
    part_off: Dict[Tuple[int, int], Tuple[int, int]] = {}  # (block sector, site state) -> (E sector, row offset)
    dims = []
    for e, mu in enumerate(mus):
        o = 0
        for st, s in enumerate(_SIGMA):
            if mu - s in lab:
                part_off[(lab[mu - s], st)] = (e, o)
                o += int(B.dims[lab[mu - s]])
        dims.append(o)
    dims = np.array(dims, np.int64)

    def build(pieces):
        """pieces: list of (block op name or None for identity, site op name, coef).
        Returns the enlarged DevOp; each piece is one dmrg_place_blocks call."""
        # destination blocks first
        keys = {}
        plans = []
        for name, sname, coef in pieces:
            items = []
            if name is None:
                blocks = [(s, s, None, int(B.dims[s]), int(B.dims[s])) for s in range(len(B.dims))]
            else:
                opb = B.ops[name]
                blocks = [(int(a), int(b), int(o), int(B.dims[b]), int(B.dims[a]))
                          for a, b, o in zip(opb.src, opb.dst, opb.off)]
            for (a, b, o, rows, cols) in blocks:  # block sector a -> b
                for (ss, sd, v) in _SITE[sname]:
                    if (a, ss) not in part_off or (b, sd) not in part_off:
                        continue
                    es, cs = part_off[(a, ss)]
                    ed, rd = part_off[(b, sd)]
                    keys.setdefault((es, ed), None)
                    items.append(((es, ed), rd, cs, rows, cols, o, coef * v))
            plans.append((name, items))
        order = sorted(keys)
        boff, pos = {}, 0
        for (es, ed) in order:
            boff[(es, ed)] = pos
            pos += int(dims[ed]) * int(dims[es])
        data = torch.zeros(max(pos, 1), dtype=torch.float64, device=dev)
        for name, items in plans:
            if not items:
                continue
            arr = (N.Place * len(items))()
            for i, ((es, ed), rd, cs, rows, cols, o, c) in enumerate(items):
                ld = int(dims[es])
                arr[i] = N.Place(0 if o is None else o, boff[(es, ed)] + rd * ld + cs, rows, cols,
                                 max(cols, 1), ld, c, 1 if o is None else 0)
            src = B.ops[name].device_data if name is not None else data
            N.check(N.lib().dmrg_place_blocks(len(items), arr, _p(src), _p(data), _stream(dev)))
        return DevOp(np.array([k[0] for k in order], np.int32), np.array([k[1] for k in order], np.int32),
                     np.array([boff[k] for k in order], np.int64), data)

    ops = {
        # H (x) I, the two spin flips and Sz (x) Sz: the last overlaps the first, so it is its own call
        "H": build([("H", "I", 1.0), ("Sp", "Sm", 0.5 * J), ("Sm", "Sp", 0.5 * J), ("Sz", "Sz", J * delta)]),
        "Sp": build([(None, "Sp", 1.0)]),
        "Sm": build([(None, "Sm", 1.0)]),
        "Sz": build([(None, "Sz", 1.0)]),
    }
    return Block(np.array(mus, np.int32), dims, ops, B.nsites + 1)


def superblock(E: Block, J: float = 1.0, delta: float = 1.0, ER: Block = None) -> _Superblock:
    """A left and a right enlarged block (the right one mirrored: its edge site
    faces the centre; ER None: the mirror image of E) coupled through their
    edge sites, S^z = 0."""
    ER = E if ER is None else ER
    sides = []
    for B in (E, ER):
        sides.append((_Space(B.labels.copy(), B.dims.copy()),
                      [_Identity(), B.ops["H"], B.ops["Sp"], B.ops["Sm"], B.ops["Sz"]]))
    terms = np.array([(1, 0), (0, 1), (2, 3), (3, 2), (4, 4)], np.int32)
    coef = np.array([1.0, 1.0, 0.5 * J, 0.5 * J, J * delta])
    return _Superblock(sides[0][0], sides[1][0], np.array([0], np.int32), sides[0][1], sides[1][1], terms, coef)


def renormalize_block(E: Block, plan, psi, m: int, side: str = "left") -> Tuple[Block, float, int]:
    """Alg. 1, steps 5-7 for one block (the enlarged block E on `side` of the
    plan's superblock): density matrix, its eigenpairs, the m kept states, and
    the operators in the kept basis."""
    import torch

    from . import eigh_blocks, renormalize, truncate

    dev = psi.device
    left = side == "left"
    rl, rr = plan.density(psi, left=left, right=not left)
    lo_l, lo_r = plan.density_layout()
    rl, lo = (rl, lo_l) if left else (rr, lo_r)
    dims = np.sqrt(np.diff(lo)).round().astype(np.int64)
    w, u, info = eigh_blocks(rl, dims, return_info=True)
    bad = info.cpu().numpy() < 0
    if bad.any():
        raise N.DmrgError(N.E_UNSUPPORTED, f"eigen-decomposition failed for blocks {np.flatnonzero(bad).tolist()}")
    keep, disc = truncate(w, dims, m)
    lay = plan.layout()
    pair_of = {int(s): k for k, s in enumerate(lay["pair_left" if left else "pair_right"])}
    kept_secs = [s for s in range(len(E.dims)) if s in pair_of and keep[pair_of[s]] > 0]
    new_index = {s: i for i, s in enumerate(kept_secs)}
    new_dims = np.array([int(keep[pair_of[s]]) for s in kept_secs], np.int64)
    ops = {}
    for name in OPS:
        op = E.ops[name]
        reqs, src, dst, off = [], [], [], []
        pos = 0
        for a, b, o in zip(op.src, op.dst, op.off):
            a, b = int(a), int(b)
            if a not in new_index or b not in new_index:
                continue
            ka, kb = int(keep[pair_of[a]]), int(keep[pair_of[b]])
            reqs.append((int(o), int(lo[pair_of[b]]), int(lo[pair_of[a]]), pos, int(E.dims[b]), int(E.dims[a]),
                         kb, ka, 0))
            src.append(new_index[a])
            dst.append(new_index[b])
            off.append(pos)
            pos += kb * ka
        data = renormalize(op.device_data, u, reqs, pos) if reqs else torch.zeros(1, dtype=torch.float64,
                                                                                 device=dev)
        ops[name] = DevOp(np.array(src, np.int32), np.array(dst, np.int32), np.array(off, np.int64), data)
    newB = Block(E.labels[kept_secs].copy(), new_dims, ops, E.nsites)
    return newB, float(disc[0]), int(new_dims.sum())


class _Workspace:
    """One caller workspace reused by the plans of consecutive steps (grown
    when a step needs more), so a step's Davidson arrays are not allocated
    again for every new superblock."""

    def __init__(self, dev, kmax):
        self.dev, self.kmax, self.buf = dev, kmax, None

    def plan(self, problem):
        import torch

        from . import Plan

        need = Plan.workspace_size(problem, "f64", self.kmax, tiles=None)
        if self.buf is None or self.buf.numel() < need:
            self.buf = None  # the previous plan is closed: its workspace may go
            self.buf = torch.empty(need + need // 4, dtype=torch.uint8, device=self.dev)
        return Plan(problem, device=self.dev, tiles=None, workspace=self.buf, ws_kmax=self.kmax)


def _solve(plan, rng, tol, kmax, kmin, use_graph=False):
    """Lowest eigenstate of the superblock (Alg. 1, step 3).  In a tiny
    superblock the preconditioned correction can fall inside the subspace
    before convergence (breakdown): then start again from another vector (at
    most three times; the count is returned and reported per step).
    Every step builds a new plan that is solved once, so by default the
    iterations are launched directly rather than captured into graphs (the
    capture would not be replayed; measured 16 % faster over a 100-site run)."""
    import torch

    for attempt in range(4):
        x0 = torch.from_numpy(rng.standard_normal(plan.n)).to(plan.device)
        psi, energy, infos, st = plan.davidson(x0, tol=tol, kmax=min(kmax, max(2, plan.n)),
                                               kmin=min(kmin, max(1, min(kmax, plan.n) - 1)),
                                               use_graph=use_graph)
        if infos[0]["converged"]:
            return psi, float(energy[0]), int(infos[0]["iterations"]), attempt
    N.check(st)
    raise N.DmrgError(N.W_NOT_CONVERGED, "Davidson did not converge")


def run_finite(nsites: int, m: int, sweeps: int = 2, J: float = 1.0, delta: float = 1.0, tol: float = 1e-10,
               device=None, seed: int = 0, kmax: int = 32, kmin: int = 8) -> Tuple[List[StepResult], List[float]]:
    """The infinite-lattice growth to `nsites`, then `sweeps` finite-lattice
    sweeps at fixed size (the optional second phase of Sec. "The DMRG
    algorithm"): the centre moves to the right end (left blocks renormalized
    from rho_L), back to the left end (right blocks from rho_R) and to the
    middle.  Returns the growth steps and the energy at the middle after each
    sweep."""
    import torch

    if nsites < 6 or nsites % 2:
        raise ValueError("nsites must be even and >= 6")
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    rng = np.random.default_rng(seed)
    L: Dict[int, Block] = {1: site_block(dev)}
    R: Dict[int, Block] = {1: L[1]}
    grow: List[StepResult] = []
    B = L[1]
    ws = _Workspace(dev, max(2, min(kmax, 48)))
    while 2 * (B.nsites + 1) <= nsites:
        E = enlarge(B, J, delta)
        plan = ws.plan(superblock(E, J, delta))
        psi, energy, its, retries = _solve(plan, rng, tol, kmax, kmin)
        B, disc, kept = renormalize_block(E, plan, psi, m)
        L[B.nsites] = R[B.nsites] = B  # mirror images of each other
        grow.append(StepResult(2 * E.nsites, energy, disc, kept, its, retries))
        plan.close()

    def step(l, side):
        r = nsites - 2 - l
        EL, ER = enlarge(L[l], J, delta), enlarge(R[r], J, delta)
        plan = ws.plan(superblock(EL, J, delta, ER))
        psi, energy, _, _ = _solve(plan, rng, tol, kmax, kmin)
        if side == "left":
            L[l + 1], _, _ = renormalize_block(EL, plan, psi, m, "left")
        else:
            R[r + 1], _, _ = renormalize_block(ER, plan, psi, m, "right")
        plan.close()
        return energy

    mid = []
    half = nsites // 2 - 1
    for _ in range(sweeps):
        for l in range(half, nsites - 3):  # centre to the right end
            step(l, "left")
        for r in range(1, nsites - 3):  # to the left end
            step(nsites - 2 - r, "right")
        e = None
        for l in range(1, half + 1):  # back to the middle (energy at l = r)
            e = step(l, "left")
        mid.append(e)
    return grow, mid


def run(nsites: int, m: int, J: float = 1.0, delta: float = 1.0, tol: float = 1e-10, device=None,
        seed: int = 0, kmax: int = 32, kmin: int = 8) -> List[StepResult]:
    """Grow the chain from 4 to `nsites` sites (even), keeping m states per
    block; returns the ground-state energy of every superblock on the way."""
    import torch

    if nsites < 4 or nsites % 2:
        raise ValueError("nsites must be even and >= 4")
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    rng = np.random.default_rng(seed)
    B = site_block(dev)
    out: List[StepResult] = []
    ws = _Workspace(dev, max(2, min(kmax, 48)))
    while 2 * (B.nsites + 1) <= nsites:
        E = enlarge(B, J, delta)
        plan = ws.plan(superblock(E, J, delta))
        psi, energy, its, retries = _solve(plan, rng, tol, kmax, kmin)
        B, disc, kept = renormalize_block(E, plan, psi, m)
        out.append(StepResult(2 * E.nsites, energy, disc, kept, its, retries))
        plan.close()
    return out
