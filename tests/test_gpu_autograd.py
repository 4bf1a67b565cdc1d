"""Energy autograd chain: backward = force kernel, double backward = HVP kernel."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_24722_amd import FP64, MIXED, workloads as W
from paper_2609_24722_amd.autograd import CoulombEnergy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-11), (MIXED, 1e-5)], ids=["fp64", "mixed"])
def test_grad_and_double_backward(dev, prec, tol):
    x, y = W.uniform_disk(500, 21)
    vx, vy = W.unit_vector(500, 22)
    xy = torch.tensor(np.stack([x, y]), device=dev, requires_grad=True)
    E = CoulombEnergy.apply(xy, prec)
    (g,) = torch.autograd.grad(E, xy, create_graph=True)
    v = torch.tensor(np.stack([vx, vy]), device=dev)
    (Hv,) = torch.autograd.grad(g, xy, v)
    fx, fy = O.forces(x, y)
    hx, hy = O.hvp(x, y, vx, vy)
    g = g.detach().cpu().numpy()
    Hv = Hv.cpu().numpy()
    assert np.linalg.norm(g - np.stack([-fx, -fy])) <= tol * np.linalg.norm(np.stack([fx, fy]))
    assert np.linalg.norm(Hv - np.stack([hx, hy])) <= tol * np.linalg.norm(np.stack([hx, hy]))
