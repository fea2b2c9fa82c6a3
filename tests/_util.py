"""Helpers shared by the tests: building surfel maps from frames with scipy's rotation
conventions (independent of both the oracle and the renderer), SE(3) perturbations and
tolerance checks."""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


def quat_wxyz(R):
    """(w, x, y, z) quaternion(s) of rotation matrix/matrices R via scipy."""
    q = Rotation.from_matrix(np.asarray(R, np.float64)).as_quat()  # scalar last
    return np.concatenate([q[..., 3:4], q[..., 0:3]], axis=-1)


def rot_of_wxyz(q):
    q = np.asarray(q, np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:4], q[..., 0:1]], axis=-1)).as_matrix()


def frame_facing(normal, spin=0.0):
    """Right-handed frame [a b n] (columns) with the given unit normal."""
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    h = np.array([0.0, 0.0, 1.0]) if abs(n[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    a = np.cross(h, n)
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    c, s = np.cos(spin), np.sin(spin)
    a, b = c * a + s * b, -s * a + c * b
    return np.stack([a, b, n], axis=1)


def surfels(centers, frames, scales, alphas):
    """float64 surfel map from centres, frames (N,3,3), scales (N,2) and opacities (N,)."""
    centers = np.asarray(centers, np.float64).reshape(-1, 3)
    frames = np.asarray(frames, np.float64).reshape(-1, 3, 3)
    scales = np.asarray(scales, np.float64).reshape(-1, 2)
    alphas = np.asarray(alphas, np.float64).reshape(-1)
    return dict(means=centers, quats=quat_wxyz(frames), log_scales=np.log(scales),
                opacity_logits=np.log(alphas) - np.log1p(-alphas))


def identity_pose():
    return np.hstack([np.eye(3), np.zeros((3, 1))])


def pose_from(R, t):
    return np.hstack([np.asarray(R, np.float64), np.asarray(t, np.float64).reshape(3, 1)])


def right_perturb(pose, xi):
    """T * Exp(xi) for a xi with only rho or only omega nonzero (exact in both cases)."""
    R, t = pose[:, :3], pose[:, 3]
    rho, om = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    Rn = R @ Rotation.from_rotvec(om).as_matrix()
    if np.any(rho != 0) and np.any(om != 0):
        raise ValueError("perturb one block at a time")
    return pose_from(Rn, t + R @ rho)


def grad_ok(g, g_ref, rel=1e-3, floor_frac=1e-3):
    """|g - g_ref| <= rel * max(|g_ref|, floor_frac * rms(g_ref)) elementwise."""
    g = np.asarray(g, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    rms = float(np.sqrt(np.mean(g_ref ** 2))) if g_ref.size else 0.0
    bound = rel * np.maximum(np.abs(g_ref), floor_frac * rms) + 1e-300
    return np.abs(g - g_ref) <= bound
