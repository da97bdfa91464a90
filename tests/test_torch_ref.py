"""The pure-PyTorch autograd reference pinned to the oracle — CPU only:
its forward intensity against ``oracle.yee.run`` and its autograd gradient
against the oracle's hand-derived reverse-mode gradient."""
import math

import numpy as np
import torch

from oracle import adjoint as OA
from oracle import problem as P
from oracle import torch_ref as T
from oracle import yee as Y
from paper_2102_12978_amd import workloads as W
from tests import cases


def _tiny():
    w = W.grad24()
    g = cases.oracle_grid(w)
    amp, ph = W.sector_params(seed=2, sectors=256)
    return w, g, amp, ph


def _loss_pieces(g, w):
    jj, ii = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    r = np.hypot(ii - g.nx / 2.0, jj + 0.5 - g.ny / 2.0)
    region = r < (w.r_outer_cells - w.thickness_cells)
    target = 2e-3 * np.exp(-(r / 3.0) ** 2)
    return region, target


def test_forward_and_gradient_match_oracle():
    w, g, amp, ph = _tiny()
    steps, wb, plane = 120, 60, g.nz // 2
    inj = cases.oracle_injector(w, amp=amp, phase=ph)
    ref = T.TorchYee(g, inj)
    a = torch.tensor(amp, requires_grad=True)
    p = torch.tensor(ph, requires_grad=True)
    ibar = ref.intensity(a, p, steps, plane, wb)
    d = Y.Diag(plane=plane, window_begin=wb)
    Y.run(g, steps, P.build_antenna(g, inj), diag=d)
    ib_o = d.mean("ey2")
    assert np.abs(ibar.detach().numpy() - ib_o).max() <= 1e-12 * np.abs(ib_o).max()
    region, target = _loss_pieces(g, w)
    reg = torch.from_numpy(region)
    loss = ((ibar - torch.from_numpy(target))[reg] ** 2).mean()
    loss.backward()
    l_o, _, ga, gp, _ = OA.intensity_loss_grad(g, inj, steps, plane, wb, target, region)
    assert abs(loss.item() - l_o) <= 1e-12 * l_o
    scale = max(np.abs(ga).max(), np.abs(gp).max())
    assert np.abs(a.grad.numpy() - ga).max() <= 1e-9 * scale
    assert np.abs(p.grad.numpy() - gp).max() <= 1e-9 * scale
    # sectors without antenna points have no gradient
    assert np.count_nonzero(ga) < 256 and np.count_nonzero(ga) > 8
