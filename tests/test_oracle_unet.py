"""Pins of the FP64 CPU U-Net reference: its autograd gradient equals central
finite differences along random directions, and the network commutes with
periodic shifts by multiples of the coarsest cell (its convolutions are
periodic and its pooling/upsampling align with that grid)."""
import numpy as np
import pytest
import torch

from oracle import unet as R

C = (16, 16, 16, 16)


def he_params(rng, c, out_ch):
    """He-scaled random parameters in the network's vector layout."""
    parts = []
    for _, ci, co in R.layer_shapes(c, out_ch):
        parts += [rng.standard_normal(co * 27 * ci) * np.sqrt(2.0 / (27 * ci)), 0.1 * rng.standard_normal(co)]
    parts += [rng.standard_normal(out_ch * c[0]) / np.sqrt(c[0]), 0.1 * rng.standard_normal(out_ch)]
    return np.concatenate(parts)


@pytest.mark.parametrize("lap_weight", [0.0, 0.5])
def test_gradient_matches_finite_differences(lap_weight):
    rng = np.random.default_rng(0)
    n, out_ch = 8, 2
    p = he_params(rng, C, out_ch)
    assert p.size == R.param_count(C, out_ch)
    x = rng.standard_normal((3, n, n, n))
    t = rng.standard_normal((out_ch, n, n, n))
    loss, g = R.loss_and_grad(p, x, t, C, out_ch, lap_weight)
    for trial in range(3):
        d = rng.standard_normal(p.shape)
        eps = 1e-6
        lp, _ = R.loss_and_grad(p + eps * d, x, t, C, out_ch, lap_weight)
        lm, _ = R.loss_and_grad(p - eps * d, x, t, C, out_ch, lap_weight)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-5 * max(1.0, abs(fd)), (fd, g @ d)


def test_periodic_shift_equivariance():
    rng = np.random.default_rng(1)
    n, out_ch = 16, 3
    p = he_params(rng, C, out_ch)
    x = rng.standard_normal((2, n, n, n))
    y = R.predict(p, x, C, out_ch)
    ys = R.predict(p, np.roll(x, (8, -8, 16), axis=(1, 2, 3)), C, out_ch)
    assert np.allclose(ys, np.roll(y, (8, -8, 16), axis=(1, 2, 3)), atol=1e-12)


def test_loss_laplacian_is_the_discrete_eigen_operator():
    """Lap of a lattice Fourier mode is the mode times sum_a (2 cos(2 pi k_a / n) - 2)."""
    n = 12
    k = (1, 3, 5)
    i = np.arange(n)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    mode = np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) / n + 0.3)
    lam = sum(2 * np.cos(2 * np.pi * ka / n) - 2 for ka in k)
    got = R.laplacian(torch.tensor(mode[None])).numpy()[0]
    assert np.abs(got - lam * mode).max() < 1e-12
