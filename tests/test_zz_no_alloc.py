"""katsevich_rmse_ssim_noscratch (the entry point for callers that cannot allocate device
memory: its reduction scratch is a library-owned static device array) against
katsevich_rmse_ssim with a caller scratch, both called through the C ABI: two calls in a
row, the second on a smaller input, each bit-identical to the caller-scratch result (same
kernels, deterministic reductions) and equal to the float64 definition of the Sec. IV
metrics to rounding."""
import ctypes

import numpy as np
import pytest

import oracle.data_oracle as DO

torch = pytest.importorskip("torch")
K = pytest.importorskip("paper_2201_02309_amd")

pytestmark = pytest.mark.gpu


def _pair(n, seed):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(0.0, 1.0, n).astype(np.float32)
    f = (ref + rng.normal(0.0, 0.05, n)).astype(np.float32)
    return f, ref


def test_noscratch_matches_caller_scratch_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    lib = K.load_library()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    nbytes = int(lib.katsevich_data_scratch_bytes())
    assert nbytes <= 164096
    for n, seed in ((3_000_017, 5), (70_001, 6)):          # second call: smaller input
        print(f"[case] rmse/ssim noscratch n={n} seed={seed}", flush=True)
        f, ref = _pair(n, seed)
        df, dref = torch.from_numpy(f).to(dev), torch.from_numpy(ref).to(dev)
        # caller scratch filled with NaN: the reduction must not read what it did not write
        scr = torch.full((nbytes // 8,), float("nan"), dtype=torch.float64, device=dev)
        r_ws = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
        r_st = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
        st = lib.katsevich_rmse_ssim(ctypes.c_void_p(df.data_ptr()), ctypes.c_void_p(dref.data_ptr()),
                                     ctypes.c_uint64(n), ctypes.c_void_p(r_ws.data_ptr()),
                                     ctypes.c_void_p(scr.data_ptr()), ctypes.c_uint64(nbytes), stream)
        assert st == 0, lib.katsevich_last_error()
        st = lib.katsevich_rmse_ssim_noscratch(ctypes.c_void_p(df.data_ptr()),
                                               ctypes.c_void_p(dref.data_ptr()), ctypes.c_uint64(n),
                                               ctypes.c_void_p(r_st.data_ptr()), stream)
        assert st == 0, lib.katsevich_last_error()
        torch.cuda.synchronize()
        a, b = r_ws.cpu().numpy(), r_st.cpu().numpy()
        print(f"[result] caller scratch {a.tolist()} static scratch {b.tolist()}", flush=True)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        want = np.array([DO.rmse(f.astype(np.float64), ref.astype(np.float64)),
                         DO.ssim(f.astype(np.float64), ref.astype(np.float64))])
        assert np.allclose(b, want, rtol=1e-10, atol=0.0), (b, want)


def test_noscratch_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = K.load_library()
    r = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = lib.katsevich_rmse_ssim_noscratch(None, None, ctypes.c_uint64(5), ctypes.c_void_p(r.data_ptr()),
                                           None)
    assert st == -1
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    st = lib.katsevich_rmse_ssim_noscratch(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_uint64(0), ctypes.c_void_p(r.data_ptr()), None)
    assert st == -1
