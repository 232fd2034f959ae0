"""The allocation-free median (hap_median_offdiag_noalloc, static device scratch) against the
allocating entry point (hap_median_offdiag), called through the C ABI: the same value bit for bit,
on two calls in a row, the second with a smaller input, in FP32 and FP64, and inside a captured
graph replayed several times."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _S(n, dt, seed):
    b = synth.small_blobs(seed, n, k=5)
    X = torch.from_numpy(b.X.astype(np.float32 if dt == torch.float32 else np.float64)).to(DEV)
    vw = 4 if dt == torch.float32 else 2
    S = torch.empty((n, n + (-n) % vw), dtype=dt, device=DEV)[:, :n]
    from paper_1403_7394_amd import hap
    hap.build_similarity(X, S)
    return S


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_noalloc_median_equals_the_allocating_call(hap_gpu, dt):
    lib = hap_gpu.load()
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    for k, n in enumerate((3001, 777)):          # the second call has a smaller input
        S = _S(n, dt, 900 + n)
        st = torch.cuda.current_stream().cuda_stream
        code = 0 if dt == torch.float32 else 1
        assert lib.hap_median_offdiag_noalloc(ctypes.c_void_p(S.data_ptr()), n, S.stride(0), code,
                                              ctypes.c_void_p(out[k:].data_ptr()), ctypes.c_void_p(st)) == 0
        torch.cuda.synchronize()
        want = ctypes.c_double()
        assert lib.hap_median_offdiag(ctypes.c_void_p(S.data_ptr()), n, S.stride(0), code, ctypes.byref(want),
                                      ctypes.c_void_p(st)) == 0
        got = float(out[k].item())
        assert np.float64(got).tobytes() == np.float64(want.value).tobytes(), (n, got, want.value)
        # the value is an off-diagonal order statistic mean: compare with a sort on the host
        v = np.sort(S.cpu().numpy()[~np.eye(n, dtype=bool)].astype(np.float64))
        ref = (v[v.size // 2 - 1] + v[v.size // 2]) / 2.0
        ref = float(np.float32(ref)) if dt == torch.float32 else ref
        assert got == ref


def test_noalloc_median_rejects_oversized_inputs_and_bad_pointers(hap_gpu):
    lib = hap_gpu.load()
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    fake = ctypes.c_void_p(4096)   # never dereferenced: the checks fail first
    assert lib.hap_median_offdiag_noalloc(fake, 65537, 65540, 0, ctypes.c_void_p(out.data_ptr()), None) == \
        hap_gpu.HAP_E_UNSUPPORTED
    assert b"65536" in lib.hap_last_error()
    assert lib.hap_median_offdiag_noalloc(fake, 100, 100, 0, None, None) == hap_gpu.HAP_E_ARG
    assert lib.hap_median_offdiag_noalloc(fake, 100, 98, 0, ctypes.c_void_p(out.data_ptr()), None) == hap_gpu.HAP_E_ARG
    assert lib.hap_median_offdiag_noalloc(fake, 100, 100, 0, ctypes.c_void_p(out.data_ptr() + 4), None) == \
        hap_gpu.HAP_E_ARG


def test_noalloc_median_replays_in_a_captured_graph(hap_gpu):
    """No allocation means the call can be captured: every replay, with eager work and a
    synchronisation between replays, gives the eager value."""
    S1, S2 = _S(1500, torch.float32, 77), _S(640, torch.float32, 78)
    want1, want2 = hap_gpu.median_offdiag(S1), hap_gpu.median_offdiag(S2)
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    hap_gpu.median_offdiag_noalloc(S1, out[0:1])    # first call on the device: outside the capture
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hap_gpu.median_offdiag_noalloc(S1, out[0:1], stream=s)
            hap_gpu.median_offdiag_noalloc(S2, out[1:2], stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert out[0].item() == want1 and out[1].item() == want2, rep
        assert hap_gpu.median_offdiag(S2) == want2     # eager work between replays
