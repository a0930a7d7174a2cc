"""The allocation-free inference call (dfhm_mlp_infer_noalloc) against
dfhm_mlp_infer, through the C ABI, on the GPU.

Both calls run the same GEMM and decode kernels on the same inputs; only the
buffers holding the hidden activations and the raw outputs differ (the
network's own against the library's static device array), so the fluxes and
error estimates must agree bit for bit.  Two calls in a row, the second with
a smaller batch, so that the second reads nothing the first left behind; a
batch above the limit is refused.
"""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bits(x):
    f = np.ascontiguousarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16).view(np.int16)


def test_noalloc_infer_matches_infer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_10119_amd import dfhm, surrogate
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(41)
    dims = (584, 512, 4, 8)
    net = surrogate.MLP(n_in=584, width=512, depth=4, n_out=8, max_batch=20000, seed=4)
    theta = mlp_ref.init(*dims[:3], seed=9, n_out=8)
    theta[-8:] = rng.normal(0, 0.2, 8)
    theta[-4:] -= 8.0
    net.set_params(theta)
    scale = np.array([0.1, 1.2, -0.3, 0.9, 1.0, 0.5, -14.0, 0.8], np.float32)
    limit = net.noalloc_max_batch()
    print(f"allocation-free limit: {limit} rows", flush=True)
    assert limit >= 20000
    for batch in (20000, 777):
        x = torch.tensor(_bits(rng.normal(0, 1, (batch, 584))), device=dev)
        f_ref, e_ref = net.infer(x, scale)
        f_na, e_na = net.infer(x, scale, noalloc=True)
        torch.cuda.synchronize()
        print(f"batch {batch}: max |flux diff| {float((f_na - f_ref).abs().max()):.3e}, "
              f"max |err diff| {float((e_na - e_ref).abs().max()):.3e}", flush=True)
        assert torch.equal(f_na, f_ref) and torch.equal(e_na, e_ref)
        assert torch.isfinite(f_na).all() and torch.isfinite(e_na).all()
    big = torch.zeros((limit + 1, 584), dtype=torch.int16, device=dev)
    with pytest.raises(dfhm.DfhmError, match="allocation-free limit"):
        net.infer(big, scale, noalloc=True)
    net.close()
