"""The bandwidth probe (hap_bandwidth_probe) computes what its mixes state, in every variant of
its access pattern (cached loads, contiguous row blocks): each output element is the sum of the
inputs at the same place, a pure write stores the row index, and the pure read leaves its sink
alone unless the data hold the marker pair."""
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("rows,cols,ld,rb,flags", [(100, 8192, 8192, 32, (False, False)), (37, 1000, 1004, 5, (False, False)),
                                                   (37, 1000, 1004, 5, (True, True)), (100, 8192, 8192, 32, (True, False)),
                                                   (100, 8192, 8192, 32, (False, True))])
def test_probe_mixes(hap_gpu, rows, cols, ld, rb, flags):
    g = torch.Generator(device="cpu").manual_seed(rows + cols)
    base = [torch.randn((rows, ld), generator=g).to(DEV) for _ in range(5)]
    cached, blocks = flags
    probe = lambda i, o, **kw: hap_gpu.bandwidth_probe(i, o, rows_per_block=rb, cached=cached, blocks=blocks, **kw)
    ins = [t[:, :cols] for t in base[:3]]
    outs = [t[:, :cols] for t in base[3:]]
    pad = [t[:, cols:].clone() for t in base[3:]]
    probe([], outs[:1])
    torch.cuda.synchronize()
    want = torch.arange(rows, dtype=torch.float32, device=DEV)[:, None].expand(rows, cols)
    assert torch.equal(outs[0], want)
    probe(ins[:1], outs[:1])
    torch.cuda.synchronize()
    assert torch.equal(outs[0], ins[0])
    probe(ins[:2], outs)
    torch.cuda.synchronize()
    s2 = ins[0] + ins[1]
    assert torch.equal(outs[0], s2) and torch.equal(outs[1], s2)
    probe(ins, outs)
    torch.cuda.synchronize()
    s3 = (ins[0] + ins[1]) + ins[2]
    assert torch.equal(outs[0], s3) and torch.equal(outs[1], s3)
    for p, t in zip(pad, base[3:]):
        assert torch.equal(t[:, cols:], p)          # the padding columns are not touched
    sink = torch.full((1,), 7.0, device=DEV)
    probe(ins[:1], [], sink=sink)
    torch.cuda.synchronize()
    assert sink.item() == 7.0


@pytest.mark.parametrize("rows,cols,ld,rb", [(100, 8192, 8192, 32), (37, 1000, 1004, 5)])
def test_probe_in_place(hap_gpu, rows, cols, ld, rb):
    """Outputs that are the last inputs (the row pass's in-place update of rho and alpha):
    every element is read before it is written, so both outputs hold the sum of the inputs'
    old values."""
    g = torch.Generator(device="cpu").manual_seed(3 * rows + cols)
    base = [torch.randn((rows, ld), generator=g).to(DEV) for _ in range(3)]
    ins = [t[:, :cols] for t in base]
    old = [t.clone() for t in ins]
    hap_gpu.bandwidth_probe(ins, ins[1:], rows_per_block=rb)
    torch.cuda.synchronize()
    s3 = (old[0] + old[1]) + old[2]
    assert torch.equal(ins[0], old[0])
    assert torch.equal(ins[1], s3) and torch.equal(ins[2], s3)
    hap_gpu.bandwidth_probe(ins[1:], ins[1:], rows_per_block=rb)
    torch.cuda.synchronize()
    assert torch.equal(ins[1], s3 + s3) and torch.equal(ins[2], s3 + s3)
