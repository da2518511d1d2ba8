"""Host logic of the inversion drivers (no GPU): the frequency-annealing
schedule (eq. fa_schedule), the positional encoding (eq. posenc_appdx), the
bounded output, and the reconstruction metrics (App. F)."""
import math

import numpy as np
import torch

from paper_2603_11045_amd.invert import InvertConfig, NeuralField, fa_weights, metrics


def test_fa_schedule_ramps_each_band_over_a_unit_interval():
    w = fa_weights(0.0, 4)
    assert torch.equal(w, torch.zeros(4, dtype=torch.float64))
    w = fa_weights(1.5, 4)                     # band 0 done, band 1 half way, bands 2, 3 off
    assert abs(w[0] - 1.0) < 1e-15 and abs(w[1] - 0.5) < 1e-15 and w[2] == 0 and w[3] == 0
    w = fa_weights(2.25, 4)
    assert abs(w[2] - 0.5 * (1 - math.cos(math.pi * 0.25))) < 1e-15
    assert torch.equal(fa_weights(4.0, 4), torch.ones(4, dtype=torch.float64))


def test_neural_field_encoding_output_bounds_and_annealing():
    cfg = InvertConfig(bands=3, depth=4, width=16, skip_layer=2, fa_horizon=10, alpha_bounds=(0.01, 0.2))
    net = NeuralField((3, 4, 5), cfg)
    assert net.coords.shape == (60, 3)
    # x runs fastest and spans [-1, 1]; the first cell sits at (-1, -1, -1)
    assert torch.allclose(net.coords[0], torch.tensor([-1.0, -1.0, -1.0]))
    assert torch.allclose(net.coords[4], torch.tensor([1.0, -1.0, -1.0]))
    assert torch.allclose(net.coords[-1], torch.tensor([1.0, 1.0, 1.0]))
    net.set_anneal(0)
    assert float(net.band_w.abs().sum()) == 0.0          # every band masked at the start
    net.set_anneal(10)
    g = net.encode()
    assert g.shape == (60, 18)
    # sin and cos of 2^k pi x for the x coordinate of cell 1 (x = -0.5)
    x = -0.5
    want = [math.sin(2 ** k * math.pi * x) for k in range(3)]
    assert np.allclose(g[1, 0:3].numpy(), want, atol=1e-6)
    with torch.no_grad():
        a = net()
    assert a.shape == (3, 4, 5)
    assert float(a.min()) > 0.01 and float(a.max()) < 0.2


def test_metrics_mse_psnr_iou():
    t = np.full((2, 3, 4), 0.15)
    t[0, 0, :2] = 0.01                          # 2 defect voxels
    a = t.copy()
    a[0, 0, 1] = 0.15                           # one missed
    a[1, 2, 3] = 0.02                           # one false
    m = metrics(a, t, bounds=(0.003, 0.25), tau=0.03)
    assert abs(m["iou"] - 1 / 3) < 1e-15
    mse = ((0.14 ** 2) + (0.13 ** 2)) / 24
    assert abs(m["mse"] - mse) < 1e-15
    assert abs(m["psnr"] - 10 * math.log10(0.247 ** 2 / mse)) < 1e-12
    assert metrics(t, t)["iou"] == 1.0
