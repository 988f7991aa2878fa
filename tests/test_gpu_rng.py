"""GPU generator parity: raw Philox words bit-exact, normals to rounding."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,level,s0,stream", [
    (1, 0, 0, 0), (1, 8, 12345, 1), ((9 << 32) | 77, 3, (5 << 32) - 100, 2), (2**64 - 1, 255, 2**40, 6)])
def test_philox_words_bit_exact(gctx, orc, torch_dev, seed, level, s0, stream):
    import torch
    nblocks, npaths = 5, 300
    out = torch.empty(npaths * nblocks * 4, dtype=torch.int32, device=torch_dev)
    gctx.mlmc_philox_words(seed, level, s0, stream, nblocks, npaths, out)
    got = out.cpu().numpy().view(np.uint32).reshape(npaths, -1)
    for i in range(0, npaths, 7):
        ref = orc.path_words(seed, level, s0 + i, stream, nblocks)
        assert np.array_equal(got[i], ref), i


@pytest.mark.parametrize("precision,dim", [(64, 1), (64, 2), (32, 1), (32, 2)])
def test_normals(gctx, orc, torch_dev, precision, dim):
    import torch
    nsteps, npaths = 37, 257
    out = torch.empty(npaths * nsteps * dim, dtype=torch.float64, device=torch_dev)
    gctx.mlmc_normals(1, 4, 1000, 0, dim, nsteps, npaths, precision, out)
    got = out.cpu().numpy().reshape(npaths, -1)
    ref = np.array([orc.path_normals(1, 4, 1000 + i, 0, dim, nsteps) for i in range(npaths)])
    err = np.abs(got - ref)
    if precision == 64:
        assert err.max() < 1e-13
    else:
        # fp32 hardware log/sqrt/sin/cos: absolute error a few 1e-7 * |z|
        assert (err / np.maximum(1, np.abs(ref))).max() < 2e-6, err.max()
