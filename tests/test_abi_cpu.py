"""Host-only checks of the C ABI: the library loads, exports every declared
entry point, and its host-side validation returns the documented status
codes without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import gen
from paper_1309_5571_amd import _native as N
from paper_1309_5571_amd import problem_check

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dmrg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmrg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = N.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(N.SIGNATURES), "binding and header disagree"


def test_version_and_default_opts():
    assert b"gfx950" in N.lib().dmrg_version()
    o = N.DavidsonOpts()
    N.lib().dmrg_davidson_default_opts(ctypes.byref(o))
    assert (o.tol, o.kmax, o.kmin, o.max_iter, o.precond_floor, o.refine, o.use_graph) == (1e-10, 32, 8, 500, 1e-3, 1, 1)


def test_struct_sizes_match_c_layout():
    assert ctypes.sizeof(N.Space) == 24
    assert ctypes.sizeof(N.Op) == 40
    assert ctypes.sizeof(N.DavidsonOpts) == 64
    assert ctypes.sizeof(N.DavidsonInfo) == 48  # two doubles, seven int32, tail padding
    assert ctypes.sizeof(N.RenormBlock) == 56
    assert ctypes.sizeof(N.Place) == 48


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_valid_problems_pass(cfg):
    assert problem_check(gen.config(cfg)) == N.OK


@pytest.mark.parametrize("seed", range(8))
def test_random_problems_pass(seed):
    assert problem_check(gen.random_problem(seed, rank=1 + seed % 2)) == N.OK


def test_unsorted_labels():
    p = gen.heisenberg_synthetic(64, seed=1)
    p.left.labels = p.left.labels[::-1].copy()
    assert problem_check(p) == N.E_LAYOUT


def test_duplicate_labels():
    p = gen.heisenberg_synthetic(64, seed=1)
    p.right.labels = p.right.labels.copy()
    p.right.labels[1] = p.right.labels[0]
    assert problem_check(p) == N.E_LAYOUT


def test_non_conserving_term():
    p = gen.heisenberg_synthetic(64, seed=1)
    p.terms = np.array([[3, 3]], dtype=np.int32)  # S+ (x) S+
    p.coef = np.array([1.0])
    assert problem_check(p) == N.E_SECTOR


def test_duplicate_block():
    p = gen.heisenberg_synthetic(64, seed=1)
    op = p.ops_left[3]
    op.src = np.concatenate([op.src, op.src[:1]])
    op.dst = np.concatenate([op.dst, op.dst[:1]])
    op.blocks = op.blocks + [op.blocks[0]]
    assert problem_check(p) == N.E_LAYOUT


def test_bad_indices():
    p = gen.heisenberg_synthetic(64, seed=1)
    p.terms = np.array([[0, 99]], dtype=np.int32)
    p.coef = np.array([1.0])
    assert problem_check(p) == N.E_INVALID_ARG
    q = gen.heisenberg_synthetic(64, seed=1)
    q.ops_left[3].src = q.ops_left[3].src.copy()
    q.ops_left[3].src[0] = 1000
    assert problem_check(q) == N.E_INVALID_ARG


def test_negative_dim_and_rank_mismatch():
    p = gen.heisenberg_synthetic(64, seed=1)
    p.left.dims = p.left.dims.copy()
    p.left.dims[0] = -1
    assert problem_check(p) == N.E_INVALID_ARG
    q = gen.hubbard_synthetic(64, seed=1)
    q.right.labels = q.right.labels[:, :1].copy()
    assert problem_check(q) in (N.E_INVALID_ARG, N.E_LAYOUT)


def test_plan_create_rejects_invalid_input_without_gpu():
    """Validation happens before any device call, so it works on a CPU host."""
    from paper_1309_5571_amd import _Marshal

    p = gen.heisenberg_synthetic(64, seed=1)
    p.terms = np.array([[3, 3]], dtype=np.int32)
    p.coef = np.array([1.0])
    m = _Marshal([p], device=None)
    h = ctypes.c_void_p()
    st = N.lib().dmrg_plan_create(ctypes.byref(h), 1, m.structs, N.F64, 0, None, 0, None)
    assert st == N.E_SECTOR and not h.value
    assert "target sector" in N.last_error()
    st = N.lib().dmrg_plan_create(ctypes.byref(h), 1, m.structs, 7, 0, None, 0, None)
    assert st == N.E_INVALID_ARG


def test_workspace_size_host_only():
    """dmrg_plan_workspace_size runs the host analysis only: it works without a
    GPU, and each extra Davidson vector adds the two basis columns (V and W,
    n doubles each) up to the 256-byte alignment of the two arrays."""
    from paper_1309_5571_amd import Plan

    p = gen.config(2)
    n = int(sum(int(p.left.dims[i]) * int(p.right.dims[j]) for i, j in _target_pairs(p)))
    sizes = {k: Plan.workspace_size(p, "f64", k) for k in (8, 9, 32, 48)}
    assert sizes[8] < sizes[9] < sizes[32] < sizes[48]
    assert abs((sizes[9] - sizes[8]) - 16 * n) <= 512
    assert abs((sizes[48] - sizes[32]) - 16 * 16 * n) <= 512
    # the reduced-precision plan may need a larger intermediate, never a smaller one
    assert Plan.workspace_size(p, "f32", 32) >= sizes[32]
    lib, m = N.lib(), _Marshal_of(p)
    b = ctypes.c_size_t()
    assert lib.dmrg_plan_workspace_size(1, m.structs, N.F64, 1, ctypes.byref(b)) == N.E_INVALID_ARG
    assert lib.dmrg_plan_workspace_size(1, m.structs, N.F64, 49, ctypes.byref(b)) == N.E_INVALID_ARG


def test_plan_create_short_workspace_is_nomem_without_gpu():
    """A workspace below the size is refused on the host (DMRG_E_NOMEM), as is
    a misaligned one (DMRG_E_INVALID_ARG); neither pointer is dereferenced."""
    from paper_1309_5571_amd import Plan

    p = gen.heisenberg_synthetic(64, seed=1)
    need = Plan.workspace_size(p, "f64", 16)
    m = _Marshal_of(p)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    st = N.lib().dmrg_plan_create(ctypes.byref(h), 1, m.structs, N.F64, 16, fake, need - 1, None)
    assert st == N.E_NOMEM and not h.value
    assert "workspace" in N.last_error()
    st = N.lib().dmrg_plan_create(ctypes.byref(h), 1, m.structs, N.F64, 16, ctypes.c_void_p((1 << 20) + 8), need, None)
    assert st == N.E_INVALID_ARG and not h.value
    st = N.lib().dmrg_plan_create(ctypes.byref(h), 1, m.structs, N.F64, 60, fake, need, None)
    assert st == N.E_INVALID_ARG


def _Marshal_of(p):
    from paper_1309_5571_amd import _Marshal

    return _Marshal([p], device=None)


def _target_pairs(p):
    """(left sector, right sector) index pairs whose labels add to the target."""
    tgt = np.asarray(p.target).reshape(-1)
    L = np.asarray(p.left.labels).reshape(len(p.left.dims), -1)
    R = np.asarray(p.right.labels).reshape(len(p.right.dims), -1)
    return [(i, j) for i in range(len(L)) for j in range(len(R)) if np.array_equal(L[i] + R[j], tgt)]


def test_gemv_argument_errors():
    lib = N.lib()
    assert lib.dmrg_gemv_t(0, 1, None, 1, None, None, None) == N.E_INVALID_ARG
    assert lib.dmrg_gemv_n(10, 65, None, 10, None, 0.0, None, None) == N.E_INVALID_ARG
    assert lib.dmrg_set_tile_table(1, (ctypes.c_int32 * 1)(8), (ctypes.c_int32 * 1)(24)) == N.E_INVALID_ARG


def test_renormalization_entry_points_validate_on_the_host():
    """Density, eigen-decomposition, selection, renormalization and placement
    reject bad arguments before any device work."""
    lib = N.lib()
    assert lib.dmrg_density(None, None, None, None, None) == N.E_INVALID_ARG
    assert lib.dmrg_density_layout(None, None, None) == N.E_INVALID_ARG
    assert lib.dmrg_eigh_blocks(-1, None, None, None, None, None, None, None, None) == N.E_INVALID_ARG
    assert lib.dmrg_eigh_blocks(0, None, None, None, None, None, None, None, None) == N.OK
    assert lib.dmrg_eigh_blocks(1, None, None, None, None, None, None, None, None) == N.E_INVALID_ARG
    fake = ctypes.c_void_p(0x1000)
    assert lib.dmrg_eigh_blocks(1, fake, fake, fake, fake, fake, fake, None, None) == N.E_INVALID_ARG  # overlap
    assert lib.dmrg_truncate(-1, None, None, None, None, None, None, None, None) == N.E_INVALID_ARG
    assert lib.dmrg_truncate(2, fake, fake, fake, fake, None, fake, None, None) == N.E_INVALID_ARG
    # renormalize: sizes and kinds are checked block by block
    a, b = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    out = ctypes.c_void_p(0x3000)
    bad = [N.RenormBlock(0, 0, 0, 0, 4, 4, 5, 4, 0),   # k_dst > rows
           N.RenormBlock(0, 0, 0, 0, 2, 3, 1, 1, 1),   # diagonal but not square
           N.RenormBlock(-1, 0, 0, 0, 2, 2, 1, 1, 0),  # negative offset
           N.RenormBlock(0, 0, 0, 0, 0, 2, 0, 1, 0),   # empty sector
           N.RenormBlock(0, 0, 0, 0, 2, 2, 1, 1, 2)]   # unknown kind
    for blk in bad:
        arr = (N.RenormBlock * 1)(blk)
        assert lib.dmrg_renormalize(1, arr, a, b, out, None) == N.E_INVALID_ARG
        assert "block 0" in N.last_error()
    ok = (N.RenormBlock * 1)(N.RenormBlock(0, 0, 0, 0, 2, 2, 1, 1, 0))
    assert lib.dmrg_renormalize(1, ok, a, b, a, None) == N.E_INVALID_ARG  # out overlaps data
    assert lib.dmrg_renormalize(-1, ok, a, b, out, None) == N.E_INVALID_ARG
    assert lib.dmrg_renormalize(0, ok, a, b, out, None) == N.OK
    # placement
    badp = [N.Place(0, 0, -1, 2, 2, 2, 1.0, 0),   # negative rows
            N.Place(0, 0, 2, 3, 3, 2, 1.0, 0),    # ld_dst < cols
            N.Place(0, 0, 2, 3, 2, 3, 1.0, 0),    # ld_src < cols
            N.Place(-4, 0, 2, 2, 2, 2, 1.0, 0),   # negative source offset
            N.Place(0, 0, 2, 2, 2, 2, 1.0, 3)]    # unknown kind
    for it in badp:
        arr = (N.Place * 1)(it)
        assert lib.dmrg_place_blocks(1, arr, a, out, None) == N.E_INVALID_ARG
    ident = (N.Place * 1)(N.Place(0, 0, 2, 2, 0, 2, 1.0, 1))
    assert lib.dmrg_place_blocks(1, ident, None, None, None) == N.E_INVALID_ARG  # null dst
    assert lib.dmrg_place_blocks(0, ident, None, None, None) == N.OK
