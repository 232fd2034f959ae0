"""Batched form: many independent problems in one persistent launch, against the oracle.

Inside the batch one workgroup owns a whole problem, so its column sums run in row order
and every problem's FP32 trajectory is the oracle's evaluated in FP32, rounding for
rounding: labels and net similarities are compared exactly (net similarity to 1e-12, the
FP64 summation order differing).
"""
import numpy as np
import pytest
import torch

from oracle import hap_ref
from oracle import similarity as sim
from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problems(sizes, d=16, seed=300):
    out = []
    for k, n in enumerate(sizes):
        b = synth.gaussian_blobs(seed + k, n, d, 3 + k % 7, centre="uniform", centre_scale=10.0, sigma_lo=1.0,
                                 sigma_hi=1.0, sizes="multinomial", dtype=np.float32)
        out.append(b.X)
    return out


def _oracle(X, L, lam, T, K=0):
    S32 = sim.similarity(X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    r = hap_ref.hap(S32, p, L, lam, T, stable_iters=K, dtype=np.float32)
    ns = [sim.net_similarity(S32, p, r.labels[l]) for l in range(L)]
    return r, ns


def _run_batch(hap, Xs, L, lam, T, K=0, launch=None):
    sizes = [x.shape[0] for x in Xs]
    X = torch.from_numpy(np.concatenate(Xs)).to(DEV)
    bt = hap.HapBatch(sizes, Xs[0].shape[1], L)
    if launch:
        bt.set_launch(*launch)
    labels, ns, iters = bt.run(X, lam, T, K)
    torch.cuda.synchronize()
    out = [bt.labels_of(labels, b).cpu().numpy() for b in range(len(sizes))], ns.cpu().numpy(), iters.cpu().numpy()
    bt.close()
    return out


def test_batch_matches_fp32_oracle_exactly(hap_gpu):
    sizes = [257, 64, 700, 2, 130, 1031, 96]
    Xs = _problems(sizes)
    L, lam, T = 3, 0.8, 30
    labels, ns, iters = _run_batch(hap_gpu, Xs, L, lam, T)
    for b, X in enumerate(Xs):
        r, ns_ref = _oracle(X, L, lam, T)
        assert np.array_equal(labels[b], r.labels), b
        assert iters[b] == T
        for l in range(L):
            assert abs(ns[b, l] - ns_ref[l]) <= 1e-12 * abs(ns_ref[l]) + 1e-300, (b, l)
        assert abs(ns[b, L] - sum(ns[b, :L])) <= 1e-12 * abs(ns[b, L])


@pytest.mark.parametrize("row_groups,threads", [(2, 512), (4, 512), (4, 1024)])
def test_batch_row_groups_match_fp32_oracle_exactly(hap_gpu, row_groups, threads):
    """Row groups sweep several rows of a problem at once; sizes cover fewer rows than
    groups, a ragged last step and the full 2048-column width."""
    sizes = [3, 5, 130, 2048, 1029]
    Xs = _problems(sizes, seed=700)
    L, lam, T = 3, 0.8, 25
    labels, ns, iters = _run_batch(hap_gpu, Xs, L, lam, T, launch=(threads, 2, row_groups))
    for b, X in enumerate(Xs):
        r, ns_ref = _oracle(X, L, lam, T)
        assert np.array_equal(labels[b], r.labels), b
        assert iters[b] == T
        for l in range(L):
            assert abs(ns[b, l] - ns_ref[l]) <= 1e-12 * abs(ns_ref[l]) + 1e-300, (b, l)


def test_batch_row_groups_stop_rule(hap_gpu):
    Xs = _problems([60, 90, 201], d=4, seed=400)
    L, lam, K = 1, 0.9, 20
    labels, ns, iters = _run_batch(hap_gpu, Xs, L, lam, 800, K, launch=(512, 3, 4))
    for b, X in enumerate(Xs):
        r, _ = _oracle(X, L, lam, 800, K)
        assert iters[b] == r.iters, b
        assert np.array_equal(labels[b], r.labels), b


def test_batch_stop_rule_matches_oracle(hap_gpu):
    Xs = _problems([60, 90, 200], d=4, seed=400)
    L, lam, K = 1, 0.9, 20
    labels, ns, iters = _run_batch(hap_gpu, Xs, L, lam, 800, K)
    for b, X in enumerate(Xs):
        r, _ = _oracle(X, L, lam, 800, K)
        assert r.converged
        assert iters[b] == r.iters, b
        assert np.array_equal(labels[b], r.labels), b


@pytest.mark.parametrize("launch", [(256, 1, 1), (512, 3, 1), (256, 1000, 1), (512, 5, 2), (512, 2, 4),
                                    (1024, 7, 4)])
def test_batch_launch_shapes_agree(hap_gpu, launch):
    """Every launch shape, row groups included, gives the same bits (the column sums of a
    problem are added in row order whatever the shape)."""
    Xs = _problems([300, 33, 1500, 64, 512], seed=500)
    base = _run_batch(hap_gpu, Xs, 3, 0.8, 12)
    got = _run_batch(hap_gpu, Xs, 3, 0.8, 12, launch=launch)
    for b in range(len(Xs)):
        assert np.array_equal(base[0][b], got[0][b])
    assert np.array_equal(base[1], got[1]) and np.array_equal(base[2], got[2])


def test_batch_graph_capture_replays(hap_gpu):
    """hap_batch_run launches kernels only, so it can be captured; every replay (with other
    GPU work and synchronisations between replays) reproduces the eager result."""
    Xs = _problems([400, 77, 1200], seed=600)
    sizes = [x.shape[0] for x in Xs]
    X = torch.from_numpy(np.concatenate(Xs)).to(DEV)
    bt = hap_gpu.HapBatch(sizes, 16, 3)
    eager = [t.clone() for t in bt.run(X, 0.8, 15)]
    torch.cuda.synchronize()
    out = bt.outputs(DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run(X, 0.8, 15, out=out, stream=s)     # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bt.run(X, 0.8, 15, out=out, stream=s)
    for _ in range(3):
        for t in out:
            t.fill_(-7) if t.dtype != torch.float64 else t.fill_(-7.0)
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b_ in zip(out, eager):
            assert torch.equal(a, b_)
        assert torch.isfinite(junk)
    bt.close()


def test_full_size_batch_on_sampled_problems(hap_gpu):
    """The batched workload at its full size (512 problems, N ~ U{64..2048}, d = 16, L = 3,
    damping 0.8) in the launch shape the benchmark's autotuner picked (1024
    threads, 512 workgroups, 4 row groups), 8 iterations: the smallest, a middle and the
    largest problem are bit-identical to the FP32 oracle (labels, and net similarity to
    1e-12); every problem reports 8 iterations and valid labels."""
    problems, rp = synth.workload_batched()
    sizes = [b.X.shape[0] for b in problems]
    X = torch.from_numpy(np.concatenate([b.X for b in problems])).to(DEV)
    bt = hap_gpu.HapBatch(sizes, 16, rp.levels)
    bt.set_launch(1024, 512, 4)
    T = 8
    labels, ns, iters = bt.run(X, rp.damping, T)
    torch.cuda.synchronize()
    assert bool(torch.all(iters == T))
    order = np.argsort(sizes, kind="stable")
    for b in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        lab = bt.labels_of(labels, b).cpu().numpy()
        assert lab.min() >= 0 and lab.max() < sizes[b]
        r, ns_ref = _oracle(problems[b].X, rp.levels, rp.damping, T)
        assert np.array_equal(lab, r.labels), (b, sizes[b])
        for l in range(rp.levels):
            assert abs(ns[b, l].item() - ns_ref[l]) <= 1e-12 * abs(ns_ref[l]), (b, l)
    bt.close()


# ---------------------------------------------------------------------------
# Problems shared by gangs of workgroups (hap_batch_set_split)
# ---------------------------------------------------------------------------

def _run_batch_split(hap, Xs, L, lam, T, split_n, max_members, K=0, launch=None, reps=1):
    sizes = [x.shape[0] for x in Xs]
    X = torch.from_numpy(np.concatenate(Xs)).to(DEV)
    bt = hap.HapBatch(sizes, Xs[0].shape[1], L)
    if launch:
        bt.set_launch(*launch)
    bt.set_split(split_n, max_members)
    members, rows = bt.members()
    outs = []
    for _ in range(reps):
        labels, ns, iters = bt.run(X, lam, T, K)
        torch.cuda.synchronize()
        outs.append(([bt.labels_of(labels, b).cpu().numpy().copy() for b in range(len(sizes))],
                     ns.cpu().numpy().copy(), iters.cpu().numpy().copy()))
    bt.close()
    return outs, members, rows


def _plain(hap, X, L, lam, T, rows_per_block, K=0):
    """The single-problem path on the same points with the given rows per workgroup, each
    workgroup taking a contiguous block of rows as a gang member does."""
    n = X.shape[0]
    Xt = torch.from_numpy(X).to(DEV)
    S = torch.empty((n, n + (-n) % 4), dtype=torch.float32, device=DEV)[:, :n]
    hap.build_similarity(Xt, S)
    h = hap.Hap(S, L, lam)
    h.set_launch(rows_per_block=rows_per_block, blocks=True)
    assert h.launch_flags() & hap.LAUNCH_BLOCKS
    res = h.iterate(T, K)
    labels = h.labels().cpu().numpy()
    ns = [h.net_similarity(l) for l in range(L)]
    h.close()
    return labels, ns, res


@pytest.mark.parametrize("L,launch", [(3, (1024, 0, 4)), (2, (512, 0, 4)), (1, (512, 0, 2))])
def test_split_problems_equal_the_plain_path_with_the_same_row_blocks(hap_gpu, L, launch):
    """A problem shared by K workgroups equals the single-problem path with rows_per_block = the
    gang's rows per member (the members' partials added in member order); problems run by one
    workgroup still equal the path with one row per workgroup.  Two levels exercise the extra
    gang barrier of that case, one level the top-level-only case."""
    sizes = [1500, 700, 300, 2048, 90, 1029]
    Xs = _problems(sizes, seed=900 + L)
    lam, T = 0.8, 25
    outs, members, rows = _run_batch_split(hap_gpu, Xs, L, lam, T, split_n=600, max_members=4,
                                           launch=(launch[0], 64, launch[2]), reps=2)
    (labels, ns, iters), (labels2, ns2, iters2) = outs
    assert members == [4, 2, 1, 4, 1, 3], members
    for b, X in enumerate(Xs):
        rb = rows[b] if members[b] > 1 else 1
        lab, ns_ref, res = _plain(hap_gpu, X, L, lam, T, rb)
        assert iters[b] == T, (b, iters[b])
        assert np.array_equal(labels[b], lab), (b, members[b])
        for l in range(L):
            assert abs(ns[b, l] - ns_ref[l]) <= 1e-12 * abs(ns_ref[l]) + 1e-300, (b, l)
        # deterministic: a second run gives the same bits
        assert np.array_equal(labels2[b], labels[b]) and np.array_equal(ns2[b], ns[b]) and iters2[b] == iters[b]


def test_split_problems_stop_rule(hap_gpu):
    """Early stops inside gangs: every member sees the OR of the members' label-change flags, so
    the stop iteration equals the single-problem path's with the same row blocks."""
    sizes = [1200, 900, 400]
    Xs = _problems(sizes, seed=950)
    L, lam, T, K = 1, 0.8, 400, 10
    outs, members, rows = _run_batch_split(hap_gpu, Xs, L, lam, T, split_n=300, max_members=8, K=K,
                                           launch=(512, 16, 4))
    labels, ns, iters = outs[0]
    assert all(k > 1 for k in members), members
    for b, X in enumerate(Xs):
        lab, ns_ref, res = _plain(hap_gpu, X, L, lam, T, rows[b], K=K)
        assert res.converged and iters[b] == res.iters, (b, iters[b], res.iters)
        assert np.array_equal(labels[b], lab), b


def test_split_plan_and_arguments(hap_gpu):
    sizes = [2048, 1024, 257, 256, 100]
    bt = hap_gpu.HapBatch(sizes, 16, 3)
    assert bt.get_split() == (0, 4) and bt.members() == ([1] * 5, sizes)
    bt.set_split(512, 8)
    k, r = bt.members()
    # K = min(8, ceil(n^2 / 512^2)) rows per member ceil(n / K); 256 points and fewer never split
    assert k == [8, 4, 1, 1, 1] and r == [256, 256, 257, 256, 100]
    for bad in ((100, 4), (512, 0), (512, 17), (-1, 4)):
        with pytest.raises(hap_gpu.HapError):
            bt.set_split(*bad)
    assert bt.get_split() == (512, 8)
    bt.set_split(0, 4)
    assert bt.members() == ([1] * 5, sizes)
    bt.close()


def test_split_full_batched_workload_sampled_problems(hap_gpu):
    """The full batched workload (512 problems, N ~ U{64..2048}, d = 16, L = 3, damping 0.8) in
    the launch and split the autotuner picks, as the benchmark does: the smallest, a middle and
    the largest problem (split, if the tuner splits it) equal the single-problem path with the
    same row blocks over 8 iterations."""
    from paper_1403_7394_amd import autotune
    problems, rp = synth.workload_batched()
    sizes = [b.X.shape[0] for b in problems]
    X = torch.from_numpy(np.concatenate([b.X for b in problems])).to(DEV)
    bt = hap_gpu.HapBatch(sizes, 16, rp.levels)
    autotune.tune_batch(bt, X, rp.damping)
    members, rows = bt.members()
    labels, ns, iters = bt.run(X, rp.damping, 8)
    torch.cuda.synchronize()
    order = np.argsort(sizes)
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    for b in picks:
        lab, ns_ref, res = _plain(hap_gpu, problems[b].X, rp.levels, rp.damping, 8,
                                  rows[b] if members[b] > 1 else 1)
        assert int(iters[b].item()) == 8
        assert np.array_equal(bt.labels_of(labels, b).cpu().numpy(), lab), (b, sizes[b], members[b])
    bt.close()
