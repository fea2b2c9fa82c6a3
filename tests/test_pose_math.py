"""Host-side pose algebra of the differentiable renderer (CPU only): the SE(3) exponential
against the matrix exponential of the twist (scipy), the right Jacobian against first-order
differences of the exponential, and the retracting pose optimiser."""
import numpy as np
import pytest
import scipy.linalg

torch = pytest.importorskip("torch")

from paper_2607_04127_amd import autograd as AG  # noqa: E402


def _twist(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = AG.hat(xi[3:])
    M[:3, 3] = xi[:3]
    return M


@pytest.mark.parametrize("scale", [0.0, 1e-7, 1e-3, 0.5, 2.5])
def test_exp_matches_matrix_exponential(scale):
    rng = np.random.default_rng(1)
    for _ in range(5):
        xi = rng.normal(size=6) * scale
        np.testing.assert_allclose(AG.se3_exp(xi), scipy.linalg.expm(_twist(xi))[:3], atol=1e-14, rtol=0)


@pytest.mark.parametrize("scale", [0.0, 1e-5, 0.3, 2.0])
def test_right_jacobian_first_order(scale):
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(4):
        xi = rng.normal(size=6) * scale
        Jr = AG.se3_right_jacobian(xi)
        for k in range(6):
            d = np.zeros(6)
            d[k] = h
            lhs = AG.se3_exp(xi + d)
            rhs = AG.compose(AG.se3_exp(xi), Jr @ d)
            assert np.abs(lhs - rhs).max() < 50 * h * h * (1 + np.linalg.norm(xi)) ** 2


def test_right_jacobian_at_zero_is_identity():
    np.testing.assert_array_equal(AG.se3_right_jacobian(np.zeros(6)), np.eye(6))


def test_compose_is_group_product():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=6) * 0.4, rng.normal(size=6) * 0.4
    T = AG.se3_exp(a)
    M = lambda X: np.vstack([X, [0, 0, 0, 1]])  # noqa: E731
    np.testing.assert_allclose(M(AG.compose(T, b)), M(T) @ M(AG.se3_exp(b)), atol=1e-14)


def test_pose_adam_retracts_into_the_base_pose():
    T0 = np.hstack([np.eye(3), np.array([[1.0], [2.0], [3.0]])])
    opt = AG.PoseAdam([T0], lr_rho=0.1, lr_omega=0.01)
    opt.xi.grad = torch.tensor([[1.0, 0, 0, 0, 0, -1.0]], dtype=torch.float64)
    opt.step()
    assert torch.all(opt.xi == 0)
    # first Adam step moves every coordinate with a nonzero gradient by -lr * sign(g)
    np.testing.assert_allclose(opt.T0[0], AG.compose(T0, np.array([-0.1, 0, 0, 0, 0, 0.01])), atol=1e-12)
