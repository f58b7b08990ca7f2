"""The allocation-free densification entry point (gb_densify_noalloc, whose work area is a
static device array) against gb_densify_plan + gb_densify_apply with a caller work buffer:
same kernels, so the outputs must be bit-identical. Two calls in a row, the second with fewer
splats (the work area keeps the first call's contents), then a call whose outputs do not fit.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FIELDS = ("means", "quats", "log_scales", "opacity_logits", "textures", "sh")
SENTINEL = -7.0


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_12734_amd import _lib as L
    return L.load()


def _inputs(P, N, seed, sh_coef=4):
    rng = np.random.default_rng(seed)
    o = rng.uniform(0.001, 0.9, P)
    host = dict(
        means=rng.uniform(-1, 1, (P, 3)), quats=rng.standard_normal((P, 4)),
        log_scales=np.log(rng.uniform(0.002, 0.05, (P, 2))), opacity_logits=np.log(o / (1 - o)),
        textures=rng.uniform(0, 1, (P, N, N, 3)), sh=rng.normal(0, 0.2, (P, sh_coef, 3)))
    dev = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in host.items()}
    accum = torch.from_numpy(rng.uniform(0, 6e-4, P).astype(np.float32)).cuda()
    vis = torch.from_numpy(rng.integers(0, 4, P).astype(np.float32)).cuda()
    noise = torch.from_numpy(rng.standard_normal((P, 2, 2)).astype(np.float32)).cuda()
    state = torch.from_numpy(rng.standard_normal((P, 7)).astype(np.float32)).cuda()
    return dev, accum, vis, noise, state


def _raw(L, t, n, N, sh_coef=4):
    return L.GbRawSplats(n, N, sh_coef, *(t[k].data_ptr() for k in FIELDS))


def _outputs(src, n):
    return {k: torch.full((n,) + tuple(v.shape[1:]), SENTINEL, dtype=torch.float32, device="cuda")
            for k, v in src.items()}


def _with_work_buffer(L, lib, P, N, src, accum, vis, noise, state, opts):
    work = torch.empty(int(lib.gb_densify_work_bytes(P)), dtype=torch.uint8, device="cuda")
    n = ctypes.c_int64(-1)
    stream = torch.cuda.current_stream().cuda_stream
    L.check(lib.gb_densify_plan(ctypes.byref(_raw(L, src, P, N)), accum.data_ptr(),
                                vis.data_ptr(), ctypes.byref(opts), work.data_ptr(), work.numel(),
                                ctypes.byref(n), stream), "gb_densify_plan")
    out = _outputs(src, n.value)
    st_out = torch.full((n.value, state.shape[1]), SENTINEL, device="cuda")
    states = (L.GbRowState * 1)(L.GbRowState(state.data_ptr(), st_out.data_ptr(), state.shape[1]))
    L.check(lib.gb_densify_apply(ctypes.byref(_raw(L, src, P, N)), work.data_ptr(),
                                 noise.data_ptr(), 0.5, ctypes.byref(opts),
                                 ctypes.byref(_raw(L, out, n.value, N)), states, 1, stream),
            "gb_densify_apply")
    torch.cuda.synchronize()
    return n.value, out, st_out


def _noalloc(L, lib, P, N, src, accum, vis, noise, state, opts, cap):
    out = _outputs(src, cap)
    st_out = torch.full((cap, state.shape[1]), SENTINEL, device="cuda")
    states = (L.GbRowState * 1)(L.GbRowState(state.data_ptr(), st_out.data_ptr(), state.shape[1]))
    n = ctypes.c_int64(-1)
    status = lib.gb_densify_noalloc(ctypes.byref(_raw(L, src, P, N)), accum.data_ptr(),
                                    vis.data_ptr(), ctypes.byref(opts), noise.data_ptr(), 0.5,
                                    ctypes.byref(_raw(L, out, cap, N)), states, 1,
                                    ctypes.byref(n), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return status, n.value, out, st_out


def _assert_rows_equal(got, want, rows):
    for k in FIELDS:
        np.testing.assert_array_equal(got[k][:rows].cpu().numpy(), want[k][:rows].cpu().numpy(),
                                      err_msg=k)


@pytest.mark.parametrize("N", [4, 8])
def test_noalloc_densify_equals_the_work_buffer_entry_points(lib, N):
    from paper_2412_12734_amd import _lib as L
    opts = L.GbDensifyOptions(2e-4, 0.01, 0.005, 0.04, 1.6)
    for P, seed in ((6000, 1), (1500, 2)):  # the second call is smaller than the first
        print(f"densify noalloc N={N} P={P} seed={seed}", flush=True)
        src, accum, vis, noise, state = _inputs(P, N, seed)
        n_ref, ref, st_ref = _with_work_buffer(L, lib, P, N, src, accum, vis, noise, state, opts)
        assert 0 < n_ref != P
        status, n, out, st_out = _noalloc(L, lib, P, N, src, accum, vis, noise, state, opts,
                                          2 * P)
        assert status == L.GB_OK and n == n_ref
        _assert_rows_equal(out, ref, n)
        np.testing.assert_array_equal(st_out[:n].cpu().numpy(), st_ref.cpu().numpy())
        # rows past the outputs are left alone
        assert bool((out["means"][n:] == SENTINEL).all())
        assert bool((st_out[n:] == SENTINEL).all())


def test_noalloc_densify_reports_outputs_that_do_not_fit(lib):
    from paper_2412_12734_amd import _lib as L
    opts = L.GbDensifyOptions(2e-4, 0.01, 0.005, 0.0, 1.6)
    P, N = 3000, 4
    src, accum, vis, noise, state = _inputs(P, N, 3)
    n_ref, ref, st_ref = _with_work_buffer(L, lib, P, N, src, accum, vis, noise, state, opts)
    cap = n_ref - 100
    status, n, out, st_out = _noalloc(L, lib, P, N, src, accum, vis, noise, state, opts, cap)
    assert status == L.GB_ERR_CAPACITY and n == n_ref
    _assert_rows_equal(out, ref, cap)
    np.testing.assert_array_equal(st_out.cpu().numpy(), st_ref[:cap].cpu().numpy())
