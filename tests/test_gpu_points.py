"""Points mode of the row pass (s_ij recomputed from the points instead of read from S)
against the same run reading S, and against the FP32 oracle: bit-identical."""
import numpy as np
import pytest
import torch

from oracle import hap_ref
from oracle import similarity as sim
from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(hap, X, L, lam, T, points, launch=None):
    n = X.shape[0]
    Xt = torch.from_numpy(X).to(DEV)
    S = torch.empty((n, n + (-n) % 4), dtype=torch.float32, device=DEV)[:, :n]
    hap.build_similarity(Xt, S)
    h = hap.Hap(S, L, lam)
    if launch:
        h.set_launch(*launch)
    if points:
        h.set_points(Xt)
    res = h.iterate(T)
    out = dict(labels=h.labels().cpu().numpy(), iters=res.iters,
               msgs=[{k: v.cpu().numpy() for k, v in h.messages(l).items()} for l in range(L)])
    h.close()
    return out


def _same(a, b, L):
    assert np.array_equal(a["labels"], b["labels"])
    for l in range(L):
        for k in ("rho", "alpha", "c", "phi"):
            assert np.array_equal(a["msgs"][l][k], b["msgs"][l][k]), (l, k)


@pytest.mark.parametrize("n,d,launch", [(1000, 2, None), (1000, 2, (256, 1, 1)), (8192, 2, None),
                                        (8192, 2, (1024, 2, 16)), (700, 3, None), (4096, 3, (512, 2, 8)),
                                        # several 64-row windows of staged per-row values per workgroup
                                        (700, 2, (256, 1, 130)), (1000, 3, (64, 4, 200)),
                                        # tiny problems: most lanes idle
                                        (2, 2, None), (5, 3, None), (65, 2, (64, 1, 65)), (129, 2, (64, 1, 3))])
def test_points_mode_equals_reading_S(hap_gpu, n, d, launch):
    b = synth.small_blobs(1200 + n + d, n, d=d, k=6, dtype=np.float32)
    L, lam, T = 3, 0.9, 12
    _same(_run(hap_gpu, b.X, L, lam, T, True, launch), _run(hap_gpu, b.X, L, lam, T, False, launch), L)


def test_points_mode_matches_fp32_oracle(hap_gpu):
    b = synth.small_blobs(1300, 600, d=2, k=5, dtype=np.float32)
    L, lam, T = 2, 0.9, 15
    g = _run(hap_gpu, b.X, L, lam, T, True, (256, 1, 1))
    S32 = sim.similarity(b.X).astype(np.float32)
    r = hap_ref.hap(S32, sim.median_offdiag(S32, np.float32), L, lam, T, dtype=np.float32)
    assert np.array_equal(g["labels"], r.labels)
    for l in range(L):
        assert np.array_equal(g["msgs"][l]["rho"], r.state.rho[l])
        assert np.array_equal(g["msgs"][l]["alpha"], r.state.alpha[l])


def test_points_mode_rejects_unsupported_inputs(hap_gpu):
    b = synth.small_blobs(1301, 100, d=4, k=3, dtype=np.float32)
    Xt = torch.from_numpy(b.X).to(DEV)
    S = torch.empty((100, 100), dtype=torch.float32, device=DEV)
    hap_gpu.build_similarity(Xt, S)
    h = hap_gpu.Hap(S, 1, 0.9)
    with pytest.raises(hap_gpu.HapError):
        h.set_points(Xt)                        # d = 4
    with pytest.raises(hap_gpu.HapError):
        h.set_points(Xt[:, :2].double())        # FP64 points
    h.close()
    S64 = S.double()
    h = hap_gpu.Hap(S64, 1, 0.9)
    with pytest.raises(hap_gpu.HapError):
        h.set_points(Xt[:, :2].contiguous())    # FP64 context
    h.close()


def test_points_mode_refuses_points_that_did_not_build_s(hap_gpu):
    """hap_set_points takes the point count and spot-checks S against X: a short X, another
    point set and another build of the same points are refused, and the context keeps
    reading S (its results equal a context that never had points set)."""
    b = synth.small_blobs(1302, 700, d=2, k=5, dtype=np.float32)
    n = b.X.shape[0]
    Xt = torch.from_numpy(b.X).to(DEV)
    S = torch.empty((n, n), dtype=torch.float32, device=DEV)
    hap_gpu.build_similarity(Xt, S)
    h = hap_gpu.Hap(S, 2, 0.9)
    with pytest.raises(hap_gpu.HapError) as e:
        h.set_points(Xt[: n - 1].contiguous())             # n - 1 points
    assert e.value.status == hap_gpu.HAP_E_ARG
    with pytest.raises(hap_gpu.HapError) as e:
        h.set_points(torch.roll(Xt, 1, dims=0).contiguous())  # the same points in another order
    assert e.value.status == hap_gpu.HAP_E_ARG
    S_gemm = torch.empty_like(S)
    hap_gpu.build_similarity(Xt, S_gemm, mode=hap_gpu.BUILD_GEMM)
    h_gemm = hap_gpu.Hap(S_gemm, 2, 0.9)
    with pytest.raises(hap_gpu.HapError) as e:
        h_gemm.set_points(Xt)                               # S from the Gram-matrix build
    assert e.value.status == hap_gpu.HAP_E_ARG
    h_gemm.close()
    h.iterate(40)
    refused = h.labels().cpu().numpy()
    h.close()
    h = hap_gpu.Hap(S, 2, 0.9)
    h.iterate(40)
    plain = h.labels().cpu().numpy()
    h.close()
    h = hap_gpu.Hap(S, 2, 0.9)
    h.set_points(Xt)                                        # the right points are accepted
    h.iterate(40)
    accepted = h.labels().cpu().numpy()
    h.close()
    assert np.array_equal(refused, plain) and np.array_equal(accepted, plain)
