"""Host logic of the autograd wrapper, checked without a GPU: a stand-in
lattice object records the calls, and the backward refuses to run when the
lattice was reused between a forward pass and its backward."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2001_11806_amd.autograd import LBMFunction  # noqa: E402


class FakeLattice:
    """Duck-typed stand-in for ``LBM`` that bumps ``generation`` on every
    trajectory-changing call exactly as the binding does."""

    def __init__(self, shape):
        self.shape = shape
        self.generation = 0
        self.calls = []

    def set_force(self, F):
        self.generation += 1
        self.calls.append("set_force")

    def init_equilibrium(self, rho, u):
        self.generation += 1
        self.calls.append("init")

    def step(self, n):
        self.generation += 1
        self.calls.append("step")

    def macroscopic(self, dtype=None):
        return None, torch.zeros(self.shape, dtype=dtype)

    def adjoint_seed(self, g):
        self.calls.append("seed")

    def adjoint_step(self, n):
        self.calls.append("adjoint_step")

    def adjoint_grads(self, dtype=None):
        return torch.ones(self.shape, dtype=dtype), None, np.zeros(3)


def _run(lat):
    u0 = torch.zeros((3, 2, 2, 2), dtype=torch.float64, requires_grad=True)
    F = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    return u0, F, LBMFunction.apply(u0, F, lat, 4)


def test_backward_runs_on_the_trajectory_of_its_forward():
    lat = FakeLattice((3, 2, 2, 2))
    u0, F, u = _run(lat)
    u.sum().backward()
    assert lat.calls == ["set_force", "init", "step", "seed", "adjoint_step"]
    assert torch.equal(u0.grad, torch.ones_like(u0))


def test_backward_after_a_second_forward_on_the_same_lattice_raises():
    lat = FakeLattice((3, 2, 2, 2))
    _, _, u_first = _run(lat)
    _run(lat)                       # overwrites the lattice's trajectory
    with pytest.raises(RuntimeError, match="no longer holds the trajectory"):
        u_first.sum().backward()
    assert "seed" not in lat.calls


def test_backward_after_stepping_the_lattice_raises():
    lat = FakeLattice((3, 2, 2, 2))
    _, _, u = _run(lat)
    lat.step(1)
    with pytest.raises(RuntimeError):
        u.sum().backward()
