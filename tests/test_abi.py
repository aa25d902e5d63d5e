"""C-ABI checks that need no GPU: the library loads, exports every function
include/fram.h declares, validates arguments before any device call, enforces
the HBM budget."""
import ctypes
import pathlib
import re

import numpy as np
import pytest

from paper_2508_00887_amd import fram as F

ROOT = pathlib.Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "fram.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fram_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = F.load_library()
    names = declared_functions()
    assert "fram_solve" in names and "fram_sdsn_project" in names and "fram_solve_many" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_declares_the_same_functions():
    assert set(declared_functions()) == set(F._SIGS)


def test_product_never_imports_the_oracle():
    for path in (ROOT / "paper_2508_00887_amd").rglob("*"):
        if path.suffix in (".py", ".hip", ".cpp", ".h"):
            src = path.read_text()
            assert "import oracle" not in src and "from oracle" not in src, path
            assert "fram64" not in src, path


@pytest.fixture
def hctx():
    c = F.Context(0)
    yield c
    c.close()


def _graph(n=6, seed=0):
    rng = np.random.default_rng(seed)
    A = np.triu(rng.random((n, n)), 1)
    return A + A.T


def _raw_solve(ctx, A, B, n, theta=2.0, iters=10, tol=0.0, opts=None):
    perm = np.zeros(max(n, 1), dtype=np.int32)
    obj = ctypes.c_double()
    st = F.Stats()
    o = opts if opts is not None else F.fram_default_options()
    a = A.ctypes.data if A is not None else None
    b = B.ctypes.data if B is not None else None
    return F.load_library().fram_solve_ex(ctx.handle, a, b, n, theta, iters, tol, ctypes.byref(o),
                                          perm.ctypes.data, ctypes.byref(obj), ctypes.byref(st))


def test_invalid_scalars_and_pointers(hctx):
    A = _graph()
    B = _graph(seed=1)
    assert _raw_solve(hctx, None, B, 6) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, None, 6) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 0) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, -3) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 6, theta=0.0) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 6, theta=-1.0) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 6, theta=float("nan")) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 6, iters=0) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 6, tol=-1e-3) == F.FRAM_EINVAL
    assert _raw_solve(hctx, A, B, 6, tol=float("inf")) == F.FRAM_EINVAL


@pytest.mark.parametrize("field,value", [("prec", 7), ("alpha", 0.0), ("alpha", 1.5),
                                         ("gamma_tol", -1.0), ("sdsn_max", 0), ("tile", 96),
                                         ("profile", 3), ("stall_iters", -1),
                                         ("stall_delta", 0.0), ("stall_delta", float("nan")),
                                         ("variant", 2), ("variant", -1), ("dsn_iters", 0),
                                         ("many_workers", 0), ("many_workers", 33),
                                         ("onchip_roll_us", -1), ("onchip_barrier_us", -5),
                                         ("onchip_barrier_us", 60000001)])
def test_invalid_options(hctx, field, value):
    o = F.fram_default_options()
    setattr(o, field, value)
    assert _raw_solve(hctx, _graph(), _graph(seed=1), 6, opts=o) == F.FRAM_EINVAL


@pytest.mark.parametrize("bad", ["negative", "nan", "inf", "asymmetric"])
def test_invalid_graph_entries(hctx, bad):
    A = _graph()
    B = _graph(seed=1)
    if bad == "negative":
        A[1, 2] = A[2, 1] = -0.5
    elif bad == "nan":
        B[0, 3] = B[3, 0] = float("nan")
    elif bad == "inf":
        B[0, 0] = float("inf")
    else:
        A[0, 1] += 1e-9
    assert _raw_solve(hctx, A, B, 6) == F.FRAM_EINVAL
    with pytest.raises(F.FramError):
        hctx.solve(A, B)


def test_budget_is_enforced_before_device_use():
    c = F.Context(0, hbm_budget_bytes=4096)
    try:
        A = _graph(100)
        assert _raw_solve(c, A, A.copy(), 100) == F.FRAM_ENOMEM
        assert "budget" in F.fram_last_error(c.handle)
    finally:
        c.close()


def test_workspace_bytes_is_monotone_and_precision_aware():
    sizes = [F.fram_workspace_bytes(n) for n in (10, 100, 1000, 4000)]
    assert sizes == sorted(sizes) and sizes[0] > 0
    assert F.fram_workspace_bytes(4000, F.FRAM_BF16) < F.fram_workspace_bytes(4000, F.FRAM_FP32)
    assert F.fram_workspace_bytes(0) == 0
    # n = 4000 needs well under 1 GB of device state.
    assert F.fram_workspace_bytes(4000, F.FRAM_FP32) < 1 << 30


def test_single_node_needs_no_device(hctx):
    perm, obj, st = hctx.solve(np.array([[3.0]]), np.array([[2.0]]))
    assert list(perm) == [0] and obj == 6.0 and st["outer_iters"] == 0


def test_create_rejects_bad_device_and_status_strings():
    h = ctypes.c_void_p()
    assert F.load_library().fram_create(ctypes.byref(h), -1, 0) == F.FRAM_EINVAL
    assert F.load_library().fram_create(None, 0, 0) == F.FRAM_EINVAL
    texts = {F.fram_status_str(s) for s in range(6)}
    assert len(texts) == 6 and "ok" in texts
    F.load_library().fram_destroy(None)


def test_solve_many_validates_every_pair(hctx):
    A = _graph()
    bad = _graph(seed=2)
    bad[0, 1] = -1.0
    with pytest.raises(F.FramError) as e:
        hctx.solve_many([A, A], [A, bad])
    assert e.value.status == F.FRAM_EINVAL


def test_sdsn_project_validates(hctx):
    K = np.ones((4, 4), dtype=np.float32)
    with pytest.raises(F.FramError):
        hctx.sdsn_project(K, theta=0.0)
    K[1, 1] = np.nan
    with pytest.raises(F.FramError):
        hctx.sdsn_project(K, theta=2.0)


def test_assign_rejects_bad_arguments_before_any_device_call(hctx):
    W = np.ones((4, 4), dtype=np.float32)
    W[2, 1] = np.inf
    with pytest.raises(F.FramError) as e:
        hctx.assign(W)
    assert e.value.status == F.FRAM_EINVAL
    lib = F.load_library()
    perm = np.zeros(4, dtype=np.int32)
    assert lib.fram_assign(hctx.handle, F._ptr(np.ones((4, 4), np.float32)), 0,
                           F._ptr(perm)) == F.FRAM_EINVAL
    assert lib.fram_assign(None, F._ptr(np.ones((4, 4), np.float32)), 4,
                           F._ptr(perm)) == F.FRAM_EINVAL
    assert lib.fram_assign_dev(hctx.handle, None, 4, 4, None, None) == F.FRAM_EINVAL
    assert lib.fram_assign_dev(hctx.handle, 1, 3, 4, 1, None) == F.FRAM_EINVAL  # ldw < n


def test_attributed_solve_rejects_bad_node_input(hctx):
    A = _graph()
    K = np.ones((6, 6))
    K[2, 3] = np.nan
    with pytest.raises(F.FramError) as e:
        hctx.solve(A, A, iters=3, K=K)
    assert e.value.status == F.FRAM_EINVAL
    with pytest.raises(F.FramError) as e:
        hctx.solve(A, A, iters=3, K=np.ones((6, 6)), node_weight=float("inf"))
    assert e.value.status == F.FRAM_EINVAL


def test_dspfp_variant_rejects_node_similarities(hctx):
    A = _graph()
    with pytest.raises(F.FramError) as e:
        hctx.solve(A, A, iters=3, K=np.ones((6, 6)), variant="dspfp")
    assert e.value.status == F.FRAM_EINVAL


def test_struct_sizes_match_the_binding():
    import ctypes
    lib = F.load_library()
    ob, sb = ctypes.c_size_t(), ctypes.c_size_t()
    lib.fram_struct_sizes(ctypes.byref(ob), ctypes.byref(sb))
    assert ob.value == ctypes.sizeof(F.Options) and sb.value == ctypes.sizeof(F.Stats)


def test_sizes_above_the_maximum_are_rejected_before_device_use(hctx):
    # FRAM_MAX_N = 32768 (32-bit element offsets of the padded FP32 iterate).
    import ctypes
    n = 32769
    A = np.zeros(1)  # never read: the size check comes first
    perm = np.zeros(1, dtype=np.int32)
    obj = ctypes.c_double()
    st = hctx.lib.fram_solve(hctx.handle, A.ctypes.data, A.ctypes.data, n, 2.0, 5, 0.0,
                             perm.ctypes.data, ctypes.byref(obj))
    assert st == F.FRAM_EINVAL
    assert hctx.lib.fram_workspace_bytes(n, 0, 0) == 0
    W = np.zeros(1, dtype=np.float32)
    assert hctx.lib.fram_assign(hctx.handle, W.ctypes.data, n, perm.ctypes.data) == F.FRAM_EINVAL


def test_warm_start_arguments_are_validated_before_device_use(hctx):
    # A non-finite host warm start is rejected on the host; fram_solve_many
    # takes no warm start or final iterate (Algorithm 1 step 1 per pair).
    A, B = _graph(), _graph(seed=1)
    N0 = np.full((6, 6), 1.0 / 6, dtype=np.float32)
    N0[2, 3] = np.nan
    o = F.fram_default_options()
    o.N0 = N0.ctypes.data
    assert _raw_solve(hctx, A, B, 6, opts=o) == F.FRAM_EINVAL
    N0[2, 3] = np.inf
    assert _raw_solve(hctx, A, B, 6, opts=o) == F.FRAM_EINVAL
    out = np.zeros((6, 6), dtype=np.float32)
    o2 = F.fram_default_options()
    o2.N_out = out.ctypes.data
    perms = [np.zeros(6, dtype=np.int32)]
    pa = (ctypes.c_void_p * 1)(A.ctypes.data)
    pb = (ctypes.c_void_p * 1)(B.ctypes.data)
    pp = (ctypes.c_void_p * 1)(perms[0].ctypes.data)
    ns = np.array([6], dtype=np.int32)
    objs = np.zeros(1)
    st = F.load_library().fram_solve_many_ex(hctx.handle, 1, pa, pb, ns.ctypes.data, 2.0, 5, 0.0,
                                             ctypes.byref(o2), pp, objs.ctypes.data, None)
    assert st == F.FRAM_EINVAL


def test_default_options_have_no_warm_start():
    o = F.fram_default_options()
    assert not o.N0 and not o.N_out


def test_noalloc_projection_validates_before_any_device_call():
    # fram_sdsn_project_noalloc: sizes above its scratch limit, the on-chip
    # mode, a tile it does not hold and NULL pointers are refused on the host.
    lib = F.load_library()
    K = np.zeros((4, 4), dtype=np.float32)
    p = K.ctypes.data

    def call(n, ldk=None, mode="stream", tile=0, dk=p, dx=p, theta=2.0):
        o = F._options("fp32", 0.95, 1e-6, 1000, tile, False, mode)
        return lib.fram_sdsn_project_noalloc(dk, ldk or n, n, theta, ctypes.byref(o), dx,
                                             ldk or n, None, None)

    assert call(1025) == F.FRAM_EINVAL            # FRAM_NOALLOC_MAX_N = 1024
    assert call(0) == F.FRAM_EINVAL
    assert call(100, ldk=99) == F.FRAM_EINVAL
    assert call(100, mode="onchip") == F.FRAM_EINVAL
    assert call(100, tile=256) == F.FRAM_EINVAL
    assert call(100, dk=None) == F.FRAM_EINVAL
    assert call(100, dx=None) == F.FRAM_EINVAL
    assert call(100, theta=0.0) == F.FRAM_EINVAL
