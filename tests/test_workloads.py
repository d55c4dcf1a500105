"""The seeded input generators: the torch form of the Gaussian field gives
the NumPy form's values bit for bit (the benchmark and the learned
correction's driver build their fields with it)."""

import numpy as np
import pytest

from paper_1606_06117_amd import workloads as W


@pytest.mark.parametrize("shape", [(24, 32, 40), (17, 9, 33), (50, 66), (64,)])
def test_random_gaussians_torch_matches_numpy(shape):
    torch = pytest.importorskip("torch")
    ref = W.random_gaussians(shape, 8, seed=2000).astype(np.float32)
    got = W.random_gaussians_torch(shape, 8, 2000, "cpu")
    assert got.dtype == torch.float32 and tuple(got.shape) == shape
    assert np.array_equal(got.numpy(), ref)


@pytest.mark.gpu
def test_random_gaussians_torch_matches_numpy_on_gpu():
    import torch
    shape = (40, 48, 72)
    ref = W.random_gaussians(shape, 8, seed=7).astype(np.float32)
    got = W.random_gaussians_torch(shape, 8, 7, "cuda").cpu().numpy()
    assert np.array_equal(got, ref)
