"""MI355X superblock projection and Davidson solver (Python binding).

A thin layer over the C ABI of ``include/dmrg.h``: it marshals problem
descriptions into the ABI structs, lets PyTorch own device memory and
streams, and wraps two entry points as ``torch.autograd.Function``s.  Every
step of the projection and of the Davidson iteration runs in the HIP
library; nothing here computes.

Problem descriptions are duck-typed: any object with the attributes
``left``/``right`` (``labels`` int [nsec, rank], ``dims`` int [nsec]),
``target``, ``ops_left``/``ops_right`` (each with ``kind`` in
{"identity", "diag", "dense"}, and ``src``/``dst``/``blocks`` or ``diag``),
``terms`` ([nterm, 2]) and ``coef`` ([nterm]).  A four-subsystem superblock
(the l-1-1-r strategy) has ``spaces`` and ``ops`` (four each: block l, site 1,
site 2, block r) and ``terms`` [nterm, 4] instead of the left/right fields.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import _native as N
from ._native import DmrgError  # noqa: F401

__all__ = ["Plan", "project", "ground_energy", "problem_check", "DmrgError", "gemv_t", "gemv_n",
           "set_tile_table", "version", "enlarge", "is_four_subsystem"]


def is_four_subsystem(p) -> bool:
    """True for a superblock given over its four subsystems (l-1-1-r)."""
    return hasattr(p, "spaces") and not hasattr(p, "left")


def version() -> str:
    return N.lib().dmrg_version().decode()


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class _Marshal:
    """Builds the ABI structs for a list of problems and keeps every buffer alive.

    ``device`` None: operator data pointers are host addresses (only valid for
    dmrg_problem_check, which never dereferences them).  Otherwise the data
    is uploaded as float64 tensors on that device.
    """

    def __init__(self, problems: Sequence, device=None):
        self.keep: list = []
        self.dev_tensors: list = []
        self.four = bool(problems) and is_four_subsystem(problems[0])
        if self.four:
            self.structs = (N.Problem4 * len(problems))()
            for i, p in enumerate(problems):
                self.structs[i] = self._problem4(p, device)
        else:
            self.structs = (N.Problem * len(problems))()
            for i, p in enumerate(problems):
                self.structs[i] = self._problem(p, device)

    def _problem4(self, p, device) -> N.Problem4:
        """Blocks l and r: data on the device (host when device is None); the
        two sites: host data, read by the library at plan creation."""
        spaces = (N.Space * 4)(*[self._space(sp) for sp in p.spaces])
        ops = (ctypes.POINTER(N.Op) * 4)()
        nop = (ctypes.c_int32 * 4)()
        for s in range(4):
            dev = device if s in (0, 3) else None
            arr = (N.Op * max(1, len(p.ops[s])))(*[self._op(o, dev) for o in p.ops[s]])
            self.keep.append(arr)
            ops[s] = ctypes.cast(arr, ctypes.POINTER(N.Op))
            nop[s] = len(p.ops[s])
        tgt = _i32(np.asarray(p.target).reshape(-1))
        t4 = _i32(np.asarray(p.terms).reshape(-1, 4))
        terms = (N.Term4 * max(1, t4.shape[0]))(*[N.Term4(*[int(x) for x in row]) for row in t4])
        self.keep += [tgt, terms, spaces, ops, nop]
        return N.Problem4(spaces, _ptr(tgt, ctypes.c_int32), nop, ops, int(t4.shape[0]), terms)

    def _space(self, sp) -> N.Space:
        lab = _i32(sp.labels)
        if lab.ndim == 1:
            lab = lab[:, None].copy()
        dims = _i64(sp.dims)
        self.keep += [lab, dims]
        return N.Space(int(dims.shape[0]), int(lab.shape[1]), _ptr(lab, ctypes.c_int32), _ptr(dims, ctypes.c_int64))

    def _data(self, arr: np.ndarray, device):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        if device is None:
            if arr.size == 0:
                arr = np.zeros(1)
            self.keep.append(arr)
            return arr.ctypes.data
        import torch

        t = torch.from_numpy(arr if arr.size else np.zeros(1)).to(device)
        self.dev_tensors.append(t)
        return t.data_ptr()

    def _op(self, op, device) -> N.Op:
        kind = N.OP_KIND[op.kind]
        if kind == N.OP_IDENTITY:
            return N.Op(kind, 0, None, None, None, None)
        if getattr(op, "device_data", None) is not None:  # dense blocks already on the device
            src, dst, off = _i32(op.src), _i32(op.dst), _i64(op.off)
            self.keep += [src, dst, off, op.device_data]
            return N.Op(kind, len(src), _ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                        _ptr(off, ctypes.c_int64), op.device_data.data_ptr())
        if kind == N.OP_DIAG:
            return N.Op(kind, 0, None, None, None, self._data(op.diag, device))
        blocks = [np.ascontiguousarray(b, dtype=np.float64) for b in op.blocks]
        sizes = np.array([b.size for b in blocks], dtype=np.int64)
        off = np.zeros(len(blocks), dtype=np.int64)
        if len(blocks) > 1:
            off[1:] = np.cumsum(sizes)[:-1]
        flat = np.concatenate([b.reshape(-1) for b in blocks]) if blocks else np.zeros(0)
        src, dst = _i32(op.src), _i32(op.dst)
        self.keep += [src, dst, off]
        return N.Op(kind, len(blocks), _ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                    _ptr(off, ctypes.c_int64), self._data(flat, device))

    def _problem(self, p, device) -> N.Problem:
        L, R = self._space(p.left), self._space(p.right)
        tgt = _i32(np.asarray(p.target).reshape(-1))
        opsL = (N.Op * max(1, len(p.ops_left)))(*[self._op(o, device) for o in p.ops_left])
        opsR = (N.Op * max(1, len(p.ops_right)))(*[self._op(o, device) for o in p.ops_right])
        terms_np = _i32(np.asarray(p.terms).reshape(-1, 2))
        terms = (N.Term * max(1, terms_np.shape[0]))(*[N.Term(int(a), int(b)) for a, b in terms_np])
        self.keep += [tgt, opsL, opsR, terms]
        return N.Problem(L, R, _ptr(tgt, ctypes.c_int32), len(p.ops_left), len(p.ops_right), opsL, opsR,
                         int(terms_np.shape[0]), terms)


def problem_check(problem) -> int:
    """Host-only validation (no GPU needed); returns the dmrg status code."""
    m = _Marshal([problem], device=None)
    return int(N.lib().dmrg_problem_check(ctypes.byref(m.structs[0])))


def set_tile_table(bounds: Sequence[int] = (), tiles: Sequence[int] = ()) -> None:
    b, t = _i32(bounds), _i32(tiles)
    N.check(N.lib().dmrg_set_tile_table(len(b), _ptr(b, ctypes.c_int32) if len(b) else None,
                                        _ptr(t, ctypes.c_int32) if len(t) else None))


def _stream(device):
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class EnlargedSpace:
    """Sector table of an enlarged block as dmrg_enlarge returns it."""

    def __init__(self, labels, dims):
        self.labels = np.ascontiguousarray(labels, dtype=np.int32)
        self.dims = np.ascontiguousarray(dims, dtype=np.int64)

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
        return np.concatenate([[0], np.cumsum(self.dims)]).astype(np.int64)


class EnlargedOp:
    """One operator of an enlarged block as dmrg_enlarge returns it (kind,
    and src/dst/blocks or diag, the layout every problem description uses)."""

    def __init__(self, kind, src=None, dst=None, blocks=None, diag=None):
        self.kind, self.src, self.dst, self.blocks, self.diag = kind, src, dst, blocks, diag

    @property
    def nblk(self) -> int:
        return len(self.blocks) if self.kind == "dense" else 0


def enlarge(slow, slow_ops, fast, fast_ops, terms, nout: int):
    """Operators of the enlarged block slow (x) fast (dmrg_enlarge, host only):
    ``terms`` = [(out, a, b, coef), ...] meaning op_out += coef *
    slow_ops[a] (x) fast_ops[b].  Returns (EnlargedSpace, [EnlargedOp] * nout)."""
    m = _Marshal([], device=None)
    S, F = m._space(slow), m._space(fast)
    os_ = (N.Op * max(1, len(slow_ops)))(*[m._op(o, None) for o in slow_ops])
    of_ = (N.Op * max(1, len(fast_ops)))(*[m._op(o, None) for o in fast_ops])
    kt = (N.KronTerm * max(1, len(terms)))(*[N.KronTerm(int(o), int(a), int(b), float(c)) for o, a, b, c in terms])
    sz = N.EnlargeSizes()
    lib = N.lib()
    args = (ctypes.byref(S), len(slow_ops), os_, ctypes.byref(F), len(fast_ops), of_, len(terms), kt, nout,
            ctypes.byref(sz))
    N.check(lib.dmrg_enlarge(*args, None, None, None, None, None, None, None, None, None))
    rank = int(np.asarray(slow.labels).reshape(slow.dims.shape[0], -1).shape[1])
    label = np.zeros(max(1, sz.nsec * rank), dtype=np.int32)
    dim = np.zeros(max(1, sz.nsec), dtype=np.int64)
    kind = np.zeros(max(1, nout), dtype=np.int32)
    nblk = np.zeros(max(1, nout), dtype=np.int32)
    ooff = np.zeros(max(1, nout), dtype=np.int64)
    src = np.zeros(max(1, sz.nblk_total), dtype=np.int32)
    dst = np.zeros(max(1, sz.nblk_total), dtype=np.int32)
    off = np.zeros(max(1, sz.nblk_total), dtype=np.int64)
    data = np.zeros(max(1, sz.data_len), dtype=np.float64)
    N.check(lib.dmrg_enlarge(*args, label.ctypes.data, dim.ctypes.data, kind.ctypes.data, nblk.ctypes.data,
                             ooff.ctypes.data, src.ctypes.data, dst.ctypes.data, off.ctypes.data,
                             data.ctypes.data))
    space = EnlargedSpace(label[:sz.nsec * rank].reshape(sz.nsec, rank), dim[:sz.nsec])
    names = {N.OP_IDENTITY: "identity", N.OP_DIAG: "diag", N.OP_DENSE: "dense"}
    ops, b = [], 0
    for o in range(nout):
        k = names[int(kind[o])]
        if k == "identity":
            ops.append(EnlargedOp("identity"))
        elif k == "diag":
            ops.append(EnlargedOp("diag", diag=data[ooff[o]:ooff[o] + sz.m].copy()))
        else:
            blocks = []
            for j in range(b, b + int(nblk[o])):
                r, c = int(dim[dst[j]]), int(dim[src[j]])
                st = int(ooff[o] + off[j])
                blocks.append(data[st:st + r * c].reshape(r, c).copy())
            ops.append(EnlargedOp("dense", src=src[b:b + nblk[o]].copy(), dst=dst[b:b + nblk[o]].copy(),
                                  blocks=blocks))
            b += int(nblk[o])
    return space, ops


class Plan:
    """A device plan for one or many superblocks (dmrg_plan_create, or
    dmrg_plan_create_l11r for superblocks given over four subsystems).

    ``prec``: "f64", "f32" or "bf16" -- the reduced precision the plan
    prepares in addition to FP64.
    ``tiles``: "auto" applies the autotuned tile table stored for this
    workload class and precision (built-in table if none is stored), None
    keeps the process-wide table as set by :func:`set_tile_table`, or a pair
    ``(bounds, tiles)`` is used for this plan only.
    ``workspace``: None (the plan allocates its scratch), a CUDA uint8 tensor
    of at least :meth:`workspace_size` bytes that the caller owns, or True (a
    tensor of that size is allocated here and kept by the plan); the scratch
    of Davidson solves with kmax <= ``ws_kmax`` then comes from it (LR plans).
    """

    @staticmethod
    def _table(problems, prec: str, tiles):
        """The tile table a plan of these problems is built with (None: the
        process-wide one)."""
        if tiles == "auto":
            if is_four_subsystem(problems[0]):
                return None
            from . import autotune

            return autotune.load_table(autotune.key_of(problems, prec))
        return tiles

    @staticmethod
    def _with_table(table, call):
        """Run call() with `table` in force (the process-wide table is restored
        after); the library's error message is read before the restore."""
        if table is None:
            st = call()
            return st, N.last_error() if st else ""
        set_tile_table(*table)
        try:
            st = call()
            msg = N.last_error() if st else ""
        finally:
            set_tile_table((), ())
        return st, msg

    @staticmethod
    def workspace_size(problems, prec: str = "f64", kmax: int = 32, tiles="auto") -> int:
        """Bytes of the caller workspace of an LR plan (dmrg_plan_workspace_size;
        host analysis only, no device call), under the tile table the plan
        will be built with (``tiles`` as in the constructor)."""
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        problems = list(problems)
        m = _Marshal(problems, device=None)
        if m.four:
            raise ValueError("plans of four subsystems (l-1-1-r) take no caller workspace")
        b = ctypes.c_size_t()
        st, msg = Plan._with_table(Plan._table(problems, prec, tiles), lambda: N.lib().dmrg_plan_workspace_size(
            len(problems), m.structs, N.PREC[prec], int(kmax), ctypes.byref(b)))
        if st:
            raise N.DmrgError(st, msg)
        return int(b.value)

    def __init__(self, problems, prec: str = "f64", device=None, tiles="auto", workspace=None, ws_kmax: int = 32):
        import torch

        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.prec = N.PREC[prec]
        self._lib = N.lib()
        self.four = is_four_subsystem(self.problems[0])
        if self.four and self.prec != N.F64:
            raise ValueError("four-subsystem (l-1-1-r) plans compute in FP64 only")
        table = Plan._table(self.problems, prec, tiles)
        self.tiles = table
        self.workspace = None
        if workspace is not None:
            if self.four:
                raise ValueError("plans of four subsystems (l-1-1-r) take no caller workspace")
            if workspace is True:
                nb = Plan.workspace_size(self.problems, prec, ws_kmax, tiles=table)
                workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
            if not (workspace.is_cuda and workspace.dtype == torch.uint8 and workspace.is_contiguous()):
                raise ValueError("workspace must be a contiguous CUDA uint8 tensor")
            self.workspace = workspace  # the caller's memory must outlive the plan
        with torch.cuda.device(self.device):
            self._m = _Marshal(self.problems, device=self.device)
            h = ctypes.c_void_p()
            ws = self.workspace
            if self.four:
                create = lambda: self._lib.dmrg_plan_create_l11r(ctypes.byref(h), len(self.problems),
                                                                 self._m.structs, _stream(self.device))
            else:
                create = lambda: self._lib.dmrg_plan_create(
                    ctypes.byref(h), len(self.problems), self._m.structs, self.prec, int(ws_kmax),
                    ws.data_ptr() if ws is not None else None, ws.numel() if ws is not None else 0,
                    _stream(self.device))
            st, msg = Plan._with_table(table, create)
            if st < 0 or st > 0:
                raise N.DmrgError(st, msg)
        self._h = h
        n, npair, nrec, flop, nbytes = (ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(),
                                        ctypes.c_int64())
        N.check(self._lib.dmrg_plan_sizes(h, ctypes.byref(n), ctypes.byref(npair), ctypes.byref(nrec),
                                          ctypes.byref(flop), ctypes.byref(nbytes)))
        self.n, self.npair, self.nrec, self.flop, self.bytes = n.value, npair.value, nrec.value, flop.value, \
            nbytes.value
        self.nterm = [int(np.asarray(p.terms).reshape(-1, 4 if self.four else 2).shape[0]) for p in self.problems]
        coef = np.concatenate([np.asarray(p.coef, dtype=np.float64).reshape(-1) for p in self.problems]) \
            if sum(self.nterm) else np.zeros(1)
        self.coef = torch.from_numpy(coef).to(self.device)
        lay = self.layout()
        self.member_off = lay["member_off"]

    # ------------------------------------------------------------ plumbing
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.dmrg_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x, name):
        import torch

        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
        if x.device != self.device:
            raise ValueError(f"{name} is on {x.device}, plan on {self.device}")
        return ctypes.c_void_p(x.data_ptr())

    def _coef(self, coef):
        c = self.coef if coef is None else coef
        if c.numel() != max(1, sum(self.nterm)):
            raise ValueError("coef has the wrong length")
        return c

    # ------------------------------------------------------------ metadata
    def layout(self) -> dict:
        np_ = self.npair
        member = np.zeros(max(np_, 1), dtype=np.int32)
        pl = np.zeros(max(np_, 1), dtype=np.int32)
        pr = np.zeros(max(np_, 1), dtype=np.int32)
        po = np.zeros(np_ + 1, dtype=np.int64)
        mo = np.zeros(len(self.problems) + 1, dtype=np.int64)
        N.check(self._lib.dmrg_plan_layout(self._h, _ptr(member, ctypes.c_int32), _ptr(pl, ctypes.c_int32),
                                           _ptr(pr, ctypes.c_int32), _ptr(po, ctypes.c_int64),
                                           _ptr(mo, ctypes.c_int64)))
        return {"member": member[:np_], "pair_left": pl[:np_], "pair_right": pr[:np_], "pair_off": po,
                "member_off": mo}

    def records(self) -> dict:
        k = max(self.nrec, 1)
        term, pin, pout, order = (np.zeros(k, dtype=np.int32) for _ in range(4))
        N.check(self._lib.dmrg_plan_records(self._h, _ptr(term, ctypes.c_int32), _ptr(pin, ctypes.c_int32),
                                            _ptr(pout, ctypes.c_int32), _ptr(order, ctypes.c_int32)))
        r = self.nrec
        return {"term": term[:r], "pair_in": pin[:r], "pair_out": pout[:r], "order": order[:r]}

    # ------------------------------------------------------------ raw entry points
    def project_raw(self, psi, coef=None, prec: str = "f64", out=None):
        import torch

        c = self._coef(coef)
        y = torch.empty_like(psi) if out is None else out
        N.check(self._lib.dmrg_project(self._h, N.PREC[prec], self._vec(c, "coef"), self._vec(psi, "psi"),
                                       self._vec(y, "y"), _stream(self.device)))
        return y

    def project_block(self, X, coef=None, out=None):
        """Y[v] = H X[v] for a [nvec, n] float64 CUDA tensor (dmrg_project_block)."""
        import torch

        c = self._coef(coef)
        if X.dim() != 2 or X.shape[1] != self.n:
            raise ValueError("X must be [nvec, n]")
        Y = torch.empty_like(X) if out is None else out
        N.check(self._lib.dmrg_project_block(self._h, X.shape[0], self._vec(c, "coef"), self._vec(X, "X"),
                                             X.stride(0), self._vec(Y, "Y"), Y.stride(0), _stream(self.device)))
        return Y

    def backward_raw(self, psi, gbar, coef=None, want_psi: bool = True, want_coef: bool = True):
        import torch

        c = self._coef(coef)
        gpsi = torch.empty_like(gbar) if want_psi else None
        gcoef = torch.empty(max(1, sum(self.nterm)), dtype=torch.float64, device=self.device) if want_coef else None
        N.check(self._lib.dmrg_project_backward(
            self._h, self._vec(c, "coef"), self._vec(psi, "psi") if want_coef else None, self._vec(gbar, "gbar"),
            self._vec(gpsi, "gpsi") if want_psi else None, self._vec(gcoef, "gcoef") if want_coef else None,
            _stream(self.device)))
        return gpsi, gcoef

    def density_layout(self) -> tuple:
        """Element offsets [npair + 1] of each pair's block in rho_left and rho_right."""
        lo = np.zeros(self.npair + 1, dtype=np.int64)
        ro = np.zeros(self.npair + 1, dtype=np.int64)
        N.check(self._lib.dmrg_density_layout(self._h, _ptr(lo, ctypes.c_int64), _ptr(ro, ctypes.c_int64)))
        return lo, ro

    def density(self, psi, left: bool = True, right: bool = True, out=None):
        """Reduced density matrices of both blocks (Alg. 1, step 5): per pair,
        Psi_p Psi_p^T and Psi_p^T Psi_p, row-major, concatenated in pair order
        (offsets from density_layout).  Either output may be skipped (None).
        out: optional (rho_left, rho_right) tensors to write into."""
        import torch

        if out is None:
            lo, ro = self.density_layout()
            rl = torch.empty(int(lo[-1]), dtype=torch.float64, device=self.device) if left else None
            rr = torch.empty(int(ro[-1]), dtype=torch.float64, device=self.device) if right else None
        else:
            rl, rr = out
            left, right = rl is not None, rr is not None
        N.check(self._lib.dmrg_density(self._h, self._vec(psi, "psi"),
                                       self._vec(rl, "rho_left") if left and rl.numel() else None,
                                       self._vec(rr, "rho_right") if right and rr.numel() else None,
                                       _stream(self.device)))
        return rl, rr

    def diagonal(self, coef=None):
        import torch

        c = self._coef(coef)
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        N.check(self._lib.dmrg_diagonal(self._h, self._vec(c, "coef"), self._vec(d, "diag"), _stream(self.device)))
        return d

    def davidson(self, psi0, coef=None, tol: float = 1e-10, kmax: int = 32, kmin: int = 8, max_iter: int = 500,
                 precond_floor: float = 1e-3, prec: str = "f64", tol_lowprec: float = 0.0, refine: bool = True,
                 use_graph: bool = True, graph_chunk: int = 8, eig_solver: str = "arrowhead",
                 raise_on_warning: bool = False):
        """Ground states of every member; returns (psi, energies [host], infos, status).
        eig_solver: "arrowhead" (direct solve of the Rayleigh step, default) or "jacobi"."""
        c = self._coef(coef)
        psi = psi0.clone()
        o = N.DavidsonOpts(tol, kmax, kmin, max_iter, precond_floor, N.PREC[prec], tol_lowprec, int(refine),
                           int(use_graph), graph_chunk, {"arrowhead": 0, "jacobi": 1}[eig_solver])
        nprob = len(self.problems)
        E = (ctypes.c_double * nprob)()
        infos = (N.DavidsonInfo * nprob)()
        st = self._lib.dmrg_davidson(self._h, self._vec(c, "coef"), ctypes.byref(o), self._vec(psi, "psi"), E,
                                     infos, _stream(self.device))
        if st < 0 and st != N.E_BREAKDOWN:
            N.check(st)
        if raise_on_warning and st != 0:
            N.check(st)
        return psi, np.array(E[:]), [infos[i].as_dict() for i in range(nprob)], int(st)


    def block_davidson(self, X0, nroots: Optional[int] = None, coef=None, tol: float = 1e-10, kmax: int = 32,
                       kmin: int = 0, max_iter: int = 500, precond_floor: float = 1e-3, chunk: int = 4):
        """The nroots lowest eigenpairs (dmrg_block_davidson).  X0: a [nroots, n]
        float64 CUDA tensor (row j = start vector j).  Returns (X [nroots, n]
        Ritz vectors, energies, residuals, info dict, status)."""
        import torch

        b = X0.shape[0] if nroots is None else nroots
        if X0.dim() != 2 or X0.shape[0] != b or X0.shape[1] != self.n:
            raise ValueError("X0 must be [nroots, n]")
        c = self._coef(coef)
        X = X0.clone().contiguous()
        o = N.BlockOpts(tol, b, kmax, kmin, max_iter, precond_floor, chunk)
        E = (ctypes.c_double * b)()
        R = (ctypes.c_double * b)()
        info = N.BlockInfo()
        st = self._lib.dmrg_block_davidson(self._h, self._vec(c, "coef"), ctypes.byref(o), self._vec(X, "X"), E, R,
                                           ctypes.byref(info), _stream(self.device))
        if st < 0:
            N.check(st)
        torch.cuda.current_stream(self.device).synchronize()
        return X, np.array(E[:]), np.array(R[:]), info.as_dict(), int(st)


# ---------------------------------------------------------------- autograd


def _torch_functions():
    import torch

    class _Project(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, psi, coef, prec):
            ctx.plan = plan
            ctx.save_for_backward(psi, coef)
            return plan.project_raw(psi.contiguous(), coef.contiguous(), prec)

        @staticmethod
        def backward(ctx, gy):
            psi, coef = ctx.saved_tensors
            gpsi, gcoef = ctx.plan.backward_raw(psi, gy.contiguous(), coef, want_psi=ctx.needs_input_grad[1],
                                                want_coef=ctx.needs_input_grad[2])
            return None, gpsi, gcoef, None

    class _GroundEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, coef, psi0, opts):
            psi, E, infos, st = plan.davidson(psi0, coef.detach().contiguous(), **opts)
            ctx.plan = plan
            ctx.save_for_backward(psi, coef)
            ctx.infos = infos
            return torch.as_tensor(E, dtype=torch.float64, device=coef.device)

        @staticmethod
        def backward(ctx, gE):
            psi, coef = ctx.saved_tensors
            # Hellmann-Feynman: dE_m / dc_k = <psi_m, T_k psi_m> for the member m owning term k
            _, gcoef = ctx.plan.backward_raw(psi, psi, coef, want_psi=False, want_coef=True)
            owner = torch.repeat_interleave(torch.arange(len(ctx.plan.nterm), device=coef.device),
                                            torch.as_tensor(ctx.plan.nterm, device=coef.device))
            return None, gcoef[: owner.numel()] * gE[owner], None, None

    return _Project, _GroundEnergy


_FN = None


def project(plan: Plan, psi, coef=None, prec: str = "f64"):
    """y = H psi, differentiable in psi and coef (backward: dmrg_project_backward)."""
    global _FN
    if _FN is None:
        _FN = _torch_functions()
    return _FN[0].apply(plan, psi, plan.coef if coef is None else coef, prec)


def ground_energy(plan: Plan, coef, psi0, **opts):
    """Lowest eigenvalue of every member, differentiable in coef (Hellmann-Feynman)."""
    global _FN
    if _FN is None:
        _FN = _torch_functions()
    return _FN[1].apply(plan, coef, psi0, opts)


def gemv_t(V, x, k: Optional[int] = None):
    """s = V[:, :k]^T x for column-major V given as a [k, n] row-per-column tensor."""
    import torch

    k = V.shape[0] if k is None else k
    s = torch.empty(k, dtype=torch.float64, device=V.device)
    N.check(N.lib().dmrg_gemv_t(V.shape[1], k, ctypes.c_void_p(V.data_ptr()), V.stride(0),
                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(s.data_ptr()), _stream(V.device)))
    return s


def gemv_n(V, s, y, beta: float = 0.0, k: Optional[int] = None):
    """y = beta y + V[:, :k] s for column-major V given as a [k, n] tensor."""
    k = V.shape[0] if k is None else k
    N.check(N.lib().dmrg_gemv_n(V.shape[1], k, ctypes.c_void_p(V.data_ptr()), V.stride(0),
                                ctypes.c_void_p(s.data_ptr()), beta, ctypes.c_void_p(y.data_ptr()),
                                _stream(V.device)))
    return y


def eigh_blocks(a, dims, return_info: bool = False):
    """Eigen-decomposition of the row-major symmetric blocks concatenated in
    `a` (orders `dims`), e.g. the output of Plan.density (Alg. 1, step 6).
    Returns (w, u): per block, eigenvalues in descending order and the
    row-major eigenvector matrix (column j for w[j]), concatenated like `a`.
    `a` is not modified (the library works on a copy)."""
    import torch

    dims = np.asarray(dims, dtype=np.int64)
    if dims.size and (dims.min() < 1 or dims.max() > 2048):
        raise ValueError("block orders must lie in 1..2048")
    off = np.zeros(dims.size, dtype=np.int64)
    woff = np.zeros(dims.size, dtype=np.int64)
    if dims.size:
        off[1:] = np.cumsum(dims * dims)[:-1]
        woff[1:] = np.cumsum(dims)[:-1]
    if a.numel() != int((dims * dims).sum()):
        raise ValueError("a does not hold the blocks")
    dev = a.device
    work = a.clone()
    w = torch.empty(int(dims.sum()), dtype=torch.float64, device=dev)
    u = torch.empty_like(a)
    t_off = torch.from_numpy(off).to(dev)
    t_dim = torch.from_numpy(dims.astype(np.int32)).to(dev)
    t_woff = torch.from_numpy(woff).to(dev)
    info = torch.zeros(max(dims.size, 1), dtype=torch.int32, device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    N.check(N.lib().dmrg_eigh_blocks(int(dims.size), p(t_off), p(t_dim), p(t_woff), p(work), p(w), p(u), p(info),
                                     _stream(dev)))
    if return_info:
        return w, u, info[: dims.size]
    return w, u


def truncate(w, dims, m_keep, groups=None):
    """Alg. 1, step 7 (state selection): keep the m_keep[g] largest of the
    eigenvalues `w` (concatenated per block, each block descending, as
    eigh_blocks returns them) in each group of consecutive blocks
    (`groups`: block counts per group; default one group).  Returns
    (kept count per block [host int array], discarded weight per group [host])."""
    import torch

    dims = np.asarray(dims, dtype=np.int64)
    groups = np.array([dims.size] if groups is None else groups, dtype=np.int64)
    if groups.sum() != dims.size or np.any(groups < 0):
        raise ValueError("groups must partition the blocks")
    m_keep = np.broadcast_to(np.asarray(m_keep, dtype=np.int32), groups.shape).copy()
    gblk = np.zeros(groups.size + 1, dtype=np.int32)
    np.cumsum(groups, out=gblk[1:])
    for g in range(groups.size):
        if int(dims[gblk[g]:gblk[g + 1]].sum()) > 16384:
            raise ValueError("a group holds more than 16384 values")
    woff = np.zeros(dims.size, dtype=np.int64)
    if dims.size:
        woff[1:] = np.cumsum(dims)[:-1]
    if w.numel() != int(dims.sum()):
        raise ValueError("w does not hold the blocks' values")
    dev = w.device
    t = lambda a: torch.from_numpy(a).to(dev)
    t_gblk, t_dim, t_woff, t_m = t(gblk), t(dims.astype(np.int32)), t(woff), t(m_keep)
    keep = torch.empty(max(dims.size, 1), dtype=torch.int32, device=dev)
    disc = torch.empty(max(groups.size, 1), dtype=torch.float64, device=dev)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    N.check(N.lib().dmrg_truncate(int(groups.size), p(t_gblk), p(t_dim), p(t_woff), p(w), p(t_m), p(keep), p(disc),
                                  _stream(dev)))
    return keep.cpu().numpy()[: dims.size], disc.cpu().numpy()[: groups.size]


def renormalize(data, u, blocks, out_len: int):
    """Alg. 1, step 7 (operators): every requested block O of `data` taken to
    the kept basis, U_dst[:, :k_dst]^T O U_src[:, :k_src], with `u` the
    eigenvector blocks from eigh_blocks.  blocks: sequence of
    (o, u_dst, u_src, out, rows, cols, k_dst, k_src, diag) element offsets and
    sizes (see dmrg_renorm_block).  Returns the output tensor of out_len."""
    import torch

    arr = (N.RenormBlock * max(len(blocks), 1))()
    for i, b in enumerate(blocks):
        arr[i] = N.RenormBlock(*[int(x) for x in b])
    out = torch.zeros(max(int(out_len), 1), dtype=torch.float64, device=data.device)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    N.check(N.lib().dmrg_renormalize(len(blocks), arr, p(data), p(u), p(out), _stream(data.device)))
    return out
