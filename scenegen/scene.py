"""Analytic scenes, virtual-scan surfel sampling, beam tables and raycast targets.

Everything here is seeded (numpy PCG64) and runs on the host in float64; arrays handed
to the renderer are float32.  Conventions (the renderer's input contract):

* beam tables: ``row_sincos[k] = (sin phi_k, cos phi_k)`` with row 0 the highest beam and
  ``phi_k = phi_max - k (phi_max - phi_min) / (H - 1)``; ``col_sincos[j] = (sin th_j, cos th_j)``
  with ``th_j = 2 pi j / W`` counter-clockwise from +x.  A pixel is one ray with direction
  ``(cos phi cos th, cos phi sin th, sin phi)`` in the sensor frame.
* pose: 3x4 row-major ``[R | t]`` mapping sensor coordinates to world coordinates.
* surfels: ``means`` (N,3) world, ``quats`` (N,4) ``(w, x, y, z)`` not normalised, whose
  rotation's columns are (major tangent, minor tangent, normal), ``log_scales`` (N,2),
  ``opacity_logits`` (N,).
* targets: ``target_depth`` (H,W) range along the ray, 0 for no return or a dropped ray;
  ``target_normal`` (H,W,3) unit surface normal in the sensor frame facing the sensor,
  zero where the depth is zero.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os

import numpy as np

GROUND_Z = -1.7


@dataclasses.dataclass
class Scene:
    # walls: rows (axis, coord, lo, hi, top) with axis 0 = plane x=coord, 1 = plane y=coord,
    # spanning [lo, hi] along the other horizontal axis and [GROUND_Z, top] in z.
    walls: np.ndarray
    # boxes: rows (x0, x1, y0, y1, z0, z1), axis aligned, standing on the ground.
    boxes: np.ndarray
    extent: tuple  # (xmin, xmax, ymin, ymax) of the walled region


# --------------------------------------------------------------------------------------
# beam model
# --------------------------------------------------------------------------------------

def beam_tables(H: int, W: int, el_min_deg: float, el_max_deg: float):
    """FP32 beam tables of a spinning LiDAR: H beams uniform in elevation (both ends
    included, row 0 on top) and W columns uniform over 360 degrees.

    Values are float64 sin/cos rounded once to float32.  When W is a multiple of 4 the
    column table is filled from its first quadrant by exact quarter-turn symmetries, so
    that a yaw of a quarter turn maps column j onto column j + W/4 exactly.
    """
    if H < 1 or W < 1:
        raise ValueError("H and W must be positive")
    phi_max = math.radians(el_max_deg)
    phi_min = math.radians(el_min_deg)
    if H == 1:
        phis = np.array([phi_max])
    else:
        k = np.arange(H, dtype=np.float64)
        phis = phi_max - k * (phi_max - phi_min) / (H - 1)
    row = np.stack([np.sin(phis), np.cos(phis)], axis=1).astype(np.float32)

    if W % 4 == 0:
        q = W // 4
        th = 2.0 * np.pi * np.arange(q, dtype=np.float64) / W
        s = np.sin(th).astype(np.float32)
        c = np.cos(th).astype(np.float32)
        col = np.empty((W, 2), np.float32)
        col[0:q, 0], col[0:q, 1] = s, c
        col[q:2 * q, 0], col[q:2 * q, 1] = c, -s
        col[2 * q:3 * q, 0], col[2 * q:3 * q, 1] = -s, -c
        col[3 * q:4 * q, 0], col[3 * q:4 * q, 1] = -c, s
    else:
        th = 2.0 * np.pi * np.arange(W, dtype=np.float64) / W
        col = np.stack([np.sin(th), np.cos(th)], axis=1).astype(np.float32)
    return np.ascontiguousarray(row), np.ascontiguousarray(col)


def ray_dirs_f64(row_sincos: np.ndarray, col_sincos: np.ndarray) -> np.ndarray:
    """(H, W, 3) float64 unit ray directions from the float32 tables (exact products)."""
    sp = row_sincos[:, 0].astype(np.float64)[:, None]
    cp = row_sincos[:, 1].astype(np.float64)[:, None]
    st = col_sincos[:, 0].astype(np.float64)[None, :]
    ct = col_sincos[:, 1].astype(np.float64)[None, :]
    H, W = sp.shape[0], st.shape[1]
    d = np.empty((H, W, 3), np.float64)
    d[..., 0] = cp * ct
    d[..., 1] = cp * st
    d[..., 2] = np.broadcast_to(sp, (H, W))
    return d


# --------------------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------------------

def _place_boxes(rng, n_boxes, extent, keep_out, margin=0.5):
    """Boxes with footprint sides U(0.5, 4) m and height U(0.5, 3) m inside ``extent``,
    none intruding within 6 m of the pose region ``keep_out`` = (xmin, xmax, ymin, ymax)."""
    xmin, xmax, ymin, ymax = extent
    kx0, kx1, ky0, ky1 = keep_out
    boxes = []
    while len(boxes) < n_boxes:
        sx, sy = rng.uniform(0.5, 4.0, size=2)
        h = rng.uniform(0.5, 3.0)
        cx = rng.uniform(xmin + margin + sx / 2, xmax - margin - sx / 2)
        cy = rng.uniform(ymin + margin + sy / 2, ymax - margin - sy / 2)
        x0, x1, y0, y1 = cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2
        # distance between the footprint rectangle and the keep-out rectangle
        dx = max(kx0 - x1, x0 - kx1, 0.0)
        dy = max(ky0 - y1, y0 - ky1, 0.0)
        if math.hypot(dx, dy) < 6.0:
            continue
        boxes.append((x0, x1, y0, y1, GROUND_Z, GROUND_Z + h))
    return np.asarray(boxes, np.float64).reshape(-1, 6)


def make_scene(kind: str, seed: int, n_boxes: int) -> Scene:
    """``room``: 4 walls at U(10, 30) m around the origin; ``block``: a 120 m x 120 m street
    block with walls at +-60 m.  Walls rise U(4, 10) m above the ground plane z = -1.7 m."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "room":
        xp, xn, yp, yn = rng.uniform(10.0, 30.0, size=4)
        extent = (-xn, xp, -yn, yp)
        keep_out = (0.0, 0.0, 0.0, 0.0)
    elif kind == "block":
        extent = (-60.0, 60.0, -60.0, 60.0)
        keep_out = (-5.0, 5.0, -5.0, 5.0)
    else:
        raise ValueError(kind)
    xmin, xmax, ymin, ymax = extent
    tops = GROUND_Z + rng.uniform(4.0, 10.0, size=4)
    walls = np.array([
        (0, xmax, ymin, ymax, tops[0]),
        (0, xmin, ymin, ymax, tops[1]),
        (1, ymax, xmin, xmax, tops[2]),
        (1, ymin, xmin, xmax, tops[3]),
    ], np.float64)
    boxes = _place_boxes(rng, n_boxes, extent, keep_out)
    return Scene(walls=walls, boxes=boxes, extent=extent)


def _raycast_chunk(scene: Scene, o: np.ndarray, d: np.ndarray):
    m = d.shape[0]
    B = scene.boxes
    best = np.full(m, np.inf)
    nrm = np.zeros((m, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        # ground plane
        tg = (GROUND_Z - o[:, 2]) / d[:, 2]
        ok = (d[:, 2] < 0) & (tg > 0)
        upd = ok & (tg < best)
        best = np.where(upd, tg, best)
        nrm[upd] = (0.0, 0.0, 1.0)
        # walls
        for axis, c, lo, hi, top in scene.walls:
            a = int(axis)
            other = 1 - a
            tw = (c - o[:, a]) / d[:, a]
            p_o = o[:, other] + tw * d[:, other]
            p_z = o[:, 2] + tw * d[:, 2]
            ok = (tw > 0) & (p_o >= lo) & (p_o <= hi) & (p_z >= GROUND_Z) & (p_z <= top)
            upd = ok & (tw < best)
            if upd.any():
                best = np.where(upd, tw, best)
                nv = np.zeros(3)
                nv[a] = 1.0
                sgn = -np.sign(d[upd, a])[:, None]
                nrm[upd] = sgn * nv[None, :]
        # boxes (slab test)
        if B.shape[0]:
            inv = 1.0 / d
            t0 = (B[None, :, 0::2] - o[:, None, :]) * inv[:, None, :]
            t1 = (B[None, :, 1::2] - o[:, None, :]) * inv[:, None, :]
            tmin = np.minimum(t0, t1)
            tent = tmin.max(axis=2)
            texit = np.maximum(t0, t1).min(axis=2)
            hit = (tent <= texit) & (tent > 0)
            tb = np.where(hit, tent, np.inf)
            jb = np.argmin(tb, axis=1)
            tbest = tb[np.arange(m), jb]
            upd = tbest < best
            if upd.any():
                rows = np.nonzero(upd)[0]
                ax = np.argmax(tmin[rows, jb[rows], :], axis=1)
                nb = np.zeros((rows.size, 3))
                nb[np.arange(rows.size), ax] = -np.sign(d[rows, ax])
                best[rows] = tbest[rows]
                nrm[rows] = nb
    hitany = np.isfinite(best)
    return np.where(hitany, best, 0.0), np.where(hitany[:, None], nrm, 0.0)


def raycast(scene: Scene, origins: np.ndarray, dirs: np.ndarray, chunk: int = 2048):
    """Nearest hit of each ray with the analytic scene, float64.

    Returns ``t`` (M,) with 0 for a miss and ``n`` (M,3) the unit surface normal facing the
    ray origin (zero for a miss).  Origins must lie above the ground and outside boxes.
    Chunks run on a thread pool (numpy releases the GIL inside its array loops)."""
    origins = np.asarray(origins, np.float64)
    dirs = np.asarray(dirs, np.float64)
    M = dirs.shape[0]
    if origins.shape[0] == 1 and M != 1:
        origins = np.broadcast_to(origins, (M, 3))
    t_out = np.zeros(M, np.float64)
    n_out = np.zeros((M, 3), np.float64)
    starts = list(range(0, M, chunk))

    def work(s):
        t, n = _raycast_chunk(scene, origins[s:s + chunk], dirs[s:s + chunk])
        t_out[s:s + t.shape[0]] = t
        n_out[s:s + t.shape[0]] = n

    nthreads = min(16, os.cpu_count() or 1, max(1, len(starts)))
    if nthreads == 1:
        for s in starts:
            work(s)
    else:
        with concurrent.futures.ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, starts))
    return t_out, n_out


def _inside_any_box(boxes, xy):
    if boxes.shape[0] == 0:
        return np.zeros(xy.shape[0], bool)
    inside = np.zeros(xy.shape[0], bool)
    for s in range(0, xy.shape[0], 4096):
        p = xy[s:s + 4096]
        inside[s:s + 4096] = ((p[:, None, 0] >= boxes[None, :, 0]) & (p[:, None, 0] <= boxes[None, :, 1])
                              & (p[:, None, 1] >= boxes[None, :, 2])
                              & (p[:, None, 1] <= boxes[None, :, 3])).any(1)
    return inside


# --------------------------------------------------------------------------------------
# surfels
# --------------------------------------------------------------------------------------

def quat_from_frame(R: np.ndarray) -> np.ndarray:
    """(w, x, y, z) unit quaternions of rotation matrices R (..., 3, 3) (Shepperd's method)."""
    R = np.asarray(R, np.float64)
    shp = R.shape[:-2]
    R = R.reshape(-1, 3, 3)
    m00, m11, m22 = R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]
    tr = m00 + m11 + m22
    q = np.empty((R.shape[0], 4))
    c0 = tr > 0
    c1 = (~c0) & (m00 >= m11) & (m00 >= m22)
    c2 = (~c0) & (~c1) & (m11 >= m22)
    c3 = (~c0) & (~c1) & (~c2)
    s = np.sqrt(np.maximum(tr[c0] + 1.0, 0)) * 2
    q[c0] = np.stack([0.25 * s, (R[c0, 2, 1] - R[c0, 1, 2]) / s, (R[c0, 0, 2] - R[c0, 2, 0]) / s,
                      (R[c0, 1, 0] - R[c0, 0, 1]) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m00[c1] - m11[c1] - m22[c1], 0)) * 2
    q[c1] = np.stack([(R[c1, 2, 1] - R[c1, 1, 2]) / s, 0.25 * s, (R[c1, 0, 1] + R[c1, 1, 0]) / s,
                      (R[c1, 0, 2] + R[c1, 2, 0]) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m11[c2] - m00[c2] - m22[c2], 0)) * 2
    q[c2] = np.stack([(R[c2, 0, 2] - R[c2, 2, 0]) / s, (R[c2, 0, 1] + R[c2, 1, 0]) / s, 0.25 * s,
                      (R[c2, 1, 2] + R[c2, 2, 1]) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m22[c3] - m00[c3] - m11[c3], 0)) * 2
    q[c3] = np.stack([(R[c3, 1, 0] - R[c3, 0, 1]) / s, (R[c3, 0, 2] + R[c3, 2, 0]) / s,
                      (R[c3, 1, 2] + R[c3, 2, 1]) / s, 0.25 * s], 1)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.reshape(shp + (4,))


def _tangent_frames(rng, normals):
    """Right-handed frames [a b n] with n given and a U(0, 2 pi) in-plane angle."""
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    helper = np.where(np.abs(n[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    a0 = np.cross(helper, n)
    a0 /= np.linalg.norm(a0, axis=1, keepdims=True)
    b0 = np.cross(n, a0)
    psi = rng.uniform(0.0, 2.0 * np.pi, size=n.shape[0])[:, None]
    a = np.cos(psi) * a0 + np.sin(psi) * b0
    b = np.cross(n, a)
    return np.stack([a, b, n], axis=2)  # columns


def _random_rotations(rng, m):
    q = rng.normal(size=(m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((m, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _pack_surfels(rng, centers, frames, ranges, delta):
    m = centers.shape[0]
    s = ranges[:, None] * delta * rng.uniform(0.8, 1.5, size=(m, 2))
    s = np.sort(s, axis=1)[:, ::-1]  # first tangent axis is the major one
    q = quat_from_frame(frames)
    # unnormalised storage with a random sign: the renderer normalises internally
    q *= (rng.uniform(0.8, 1.25, size=m) * rng.choice([-1.0, 1.0], size=m))[:, None]
    alpha = rng.uniform(0.3, 0.95, size=m)
    logit = np.log(alpha) - np.log1p(-alpha)
    return dict(means=centers.astype(np.float32), quats=q.astype(np.float32),
                log_scales=np.log(s).astype(np.float32), opacity_logits=logit.astype(np.float32))


def sample_surfels(scene: Scene, n: int, seed: int, el_range_deg, delta: float, r_max: float,
                   origin_mode: str, rays_per_origin: int = 64, blob_fraction: float = 0.0,
                   blob_radius: float = 0.5, n_blobs: int = 0):
    """Surfels from virtual scans: random rays (azimuth U(0, 2 pi), elevation uniform over
    ``el_range_deg``) from sampling origins at z = 0; hits with range in [2, r_max] become
    surfel centres with the surface normal facing the origin, a random in-plane angle,
    tangent scales ``r * delta * U(0.8, 1.5)`` and opacity U(0.3, 0.95).

    ``origin_mode``: ``"origin"`` samples from (0, 0, 0) only; ``"block"`` draws origins
    uniformly over [-50, 50]^2 outside boxes.  A ``blob_fraction`` of the surfels are placed
    in ``n_blobs`` balls of radius ``blob_radius`` centred on surface points, with uniformly
    random orientation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    el0, el1 = math.radians(el_range_deg[0]), math.radians(el_range_deg[1])
    n_blob_members = int(round(n * blob_fraction)) if n_blobs > 0 else 0
    n_surf = n - n_blob_members
    need = n_surf + n_blobs
    centers, normals, ranges = [], [], []
    got = 0
    while got < need:
        batch = max(4096, int((need - got) * 1.6))
        n_or = max(1, batch // rays_per_origin)
        if origin_mode == "origin":
            o = np.zeros((n_or, 3))
        else:
            o = np.zeros((0, 3))
            while o.shape[0] < n_or:
                cand = np.zeros((n_or, 3))
                cand[:, :2] = rng.uniform(-50.0, 50.0, size=(n_or, 2))
                cand = cand[~_inside_any_box(scene.boxes, cand[:, :2])]
                o = np.concatenate([o, cand])[:n_or]
        o = np.repeat(o, rays_per_origin, axis=0)
        m = o.shape[0]
        az = rng.uniform(0.0, 2.0 * np.pi, size=m)
        el = rng.uniform(el0, el1, size=m)
        d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], 1)
        t, nrm = raycast(scene, o, d)
        keep = (t >= 2.0) & (t <= r_max)
        p = o[keep] + t[keep, None] * d[keep]
        centers.append(p)
        normals.append(nrm[keep])
        ranges.append(t[keep])
        got += int(keep.sum())
    centers = np.concatenate(centers)[:need]
    normals = np.concatenate(normals)[:need]
    ranges = np.concatenate(ranges)[:need]

    surf_c, surf_n, surf_r = centers[:n_surf], normals[:n_surf], ranges[:n_surf]
    frames = _tangent_frames(rng, surf_n)
    out = _pack_surfels(rng, surf_c, frames, surf_r, delta)
    if n_blob_members:
        bc, br = centers[n_surf:], ranges[n_surf:]
        which = rng.integers(0, n_blobs, size=n_blob_members)
        v = rng.normal(size=(n_blob_members, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        rad = blob_radius * rng.uniform(0.0, 1.0, size=n_blob_members) ** (1.0 / 3.0)
        pc = bc[which] + rad[:, None] * v
        fb = _random_rotations(rng, n_blob_members)
        blob = _pack_surfels(rng, pc, fb, br[which], delta)
        out = {k: np.concatenate([out[k], blob[k]]) for k in out}
    return out


# --------------------------------------------------------------------------------------
# poses and targets
# --------------------------------------------------------------------------------------

def make_pose(yaw: float, tx: float, ty: float, tz: float = 0.0) -> np.ndarray:
    """3x4 float32 sensor-to-world pose with a yaw rotation about +z."""
    c, s = math.cos(yaw), math.sin(yaw)
    P = np.array([[c, -s, 0.0, tx], [s, c, 0.0, ty], [0.0, 0.0, 1.0, tz]], np.float64)
    return P.astype(np.float32)


def targets_for_pose(scene: Scene, pose: np.ndarray, row_sincos, col_sincos,
                     drop_rate: float = 0.0, drop_seed: int = 0):
    """Exact raycast of the analytic scene from ``pose`` along every beam.  Returns the
    float32 target range image (H,W) and sensor-frame normals (H,W,3), with a Bernoulli
    ``drop_rate`` of rays zeroed (no return)."""
    P = np.asarray(pose, np.float64)
    R, t = P[:, :3], P[:, 3]
    d = ray_dirs_f64(row_sincos, col_sincos)
    H, W = d.shape[:2]
    dw = d.reshape(-1, 3) @ R.T
    tt, nw = raycast(scene, t[None, :], dw)
    ns = nw @ R  # world -> sensor: R^T n, row-vector form
    depth = tt.reshape(H, W)
    normal = ns.reshape(H, W, 3)
    if drop_rate > 0:
        rng = np.random.Generator(np.random.PCG64(drop_seed))
        drop = rng.uniform(size=(H, W)) < drop_rate
        depth = np.where(drop, 0.0, depth)
        normal = np.where(drop[..., None], 0.0, normal)
    return depth.astype(np.float32), normal.astype(np.float32)


def synthetic_frame(scene: Scene, pose: np.ndarray, row_sincos, col_sincos, seed: int,
                    range_noise: float = 0.01, hole_rate: float = 0.05):
    """A frame shaped like a renderer's output, for tests of the loss: depth = exact raycast
    times (1 + N(0, range_noise)) with a Bernoulli hole_rate of rays and every no-return ray
    zero; opacity U(0.3, 1) on rays with a depth, else 0; normal = the raycast normal
    (sensor frame) plus N(0, 0.05) noise, scaled by the opacity.  float32 arrays (H,W),
    (H,W), (H,W,3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    depth, normal = targets_for_pose(scene, pose, row_sincos, col_sincos)
    H, W = depth.shape
    d = depth.astype(np.float64) * (1.0 + rng.normal(0.0, range_noise, size=(H, W)))
    d[(rng.uniform(size=(H, W)) < hole_rate) | ~(depth > 0)] = 0.0
    op = np.where(d > 0, rng.uniform(0.3, 1.0, size=(H, W)), 0.0)
    nrm = (normal.astype(np.float64) + rng.normal(0.0, 0.05, size=(H, W, 3))) * op[..., None]
    return d.astype(np.float32), op.astype(np.float32), nrm.astype(np.float32)


def synthetic_scan(scene: Scene, pose: np.ndarray, H: int, W: int, el_min_deg: float, el_max_deg: float,
                   seed: int, az_jitter: float = 0.3, el_jitter: float = 0.05, extra_fraction: float = 0.2,
                   range_noise: float = 0.01):
    """A spinning-LiDAR scan of the scene in the sensor frame: one ray per beam and column,
    azimuth jittered by U(-az_jitter, az_jitter) of a column and elevation by
    U(-el_jitter, el_jitter) of a row, range = exact raycast times (1 + N(0, range_noise)),
    returns beyond the scene dropped; plus extra_fraction more points as second returns in
    front of the first along random rays (a partial occluder between 20% and 95% of the
    range).  Normals: the surface normals at the hits with random signs (the orientation a
    covariance's principal axis has).  float32 (n, 3) points and normals, shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = np.asarray(pose, np.float64)
    R, t = P[:, :3], P[:, 3]
    phi_max, phi_min = math.radians(el_max_deg), math.radians(el_min_deg)
    k = np.repeat(np.arange(H), W).astype(np.float64)
    j = np.tile(np.arange(W), H).astype(np.float64)
    el = phi_max - (k + rng.uniform(-el_jitter, el_jitter, k.size)) * (phi_max - phi_min) / max(H - 1, 1)
    az = 2.0 * np.pi * (j + rng.uniform(-az_jitter, az_jitter, j.size)) / W
    d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], 1)
    tt, nw = raycast(scene, np.broadcast_to(t, d.shape), d @ R.T)
    keep = np.isfinite(tt) & (tt > 0)
    r = tt[keep] * (1.0 + rng.normal(0.0, range_noise, keep.sum()))
    pts = r[:, None] * d[keep]
    nrm = (nw[keep] @ R) * rng.choice([-1.0, 1.0], size=(keep.sum(), 1))
    m = int(round(extra_fraction * pts.shape[0]))
    if m:
        src = rng.integers(0, pts.shape[0], m)
        pts = np.concatenate([pts, pts[src] * rng.uniform(0.2, 0.95, (m, 1))])
        v = rng.normal(size=(m, 3))
        nrm = np.concatenate([nrm, v / np.linalg.norm(v, axis=1, keepdims=True)])
    perm = rng.permutation(pts.shape[0])
    return pts[perm].astype(np.float32), nrm[perm].astype(np.float32)


# --------------------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------------------

WORKLOADS = {
    # 32x256 beams over +-15 deg, 1,000 surfels in a 4-wall room with 20 boxes, identity pose.
    "room32x256_1k": dict(index=1, H=32, W=256, el=(-15.0, 15.0), n=1000, kind="room", n_boxes=20,
                          r_max=40.0, origin_mode="origin", pose="identity", drop=0.0),
    # 64x1024 beams over +-22.5 deg, 300,000 surfels in a 120 m street block with 400 boxes,
    # random yaw and +-5 m translation, 10% of rays dropped.
    "block64x1024_300k": dict(index=2, H=64, W=1024, el=(-22.5, 22.5), n=300_000, kind="block",
                              n_boxes=400, r_max=40.0, origin_mode="block", pose="random", drop=0.1),
    # 64x2048 beams over -24.9..+2.0 deg, 1M surfels, 8 poses 1.5 m apart with yaw noise.
    "window64x2048_1m": dict(index=3, H=64, W=2048, el=(-24.9, 2.0), n=1_000_000, kind="block",
                             n_boxes=400, r_max=40.0, origin_mode="block", pose="trajectory",
                             n_poses=8, drop=0.0),
    # 128x2048 beams over +-45 deg, 4M surfels, 30% of them in 0.5 m blobs.
    "deep128x2048_4m": dict(index=5, H=128, W=2048, el=(-45.0, 45.0), n=4_000_000, kind="block",
                            n_boxes=400, r_max=40.0, origin_mode="block", pose="random", drop=0.0,
                            blob_fraction=0.3, n_blobs=2000),
}


def make_workload(name: str, n: int | None = None, H: int | None = None, W: int | None = None,
                  with_targets: bool = True):
    """Build a named workload (optionally overriding N, H, W) with seeds scene = K,
    pose = 100 + K, drop = 200 + K for workload index K."""
    cfg = dict(WORKLOADS[name])
    K = cfg["index"]
    if n is not None:
        cfg["n"] = n
    if H is not None:
        cfg["H"] = H
    if W is not None:
        cfg["W"] = W
    H_, W_ = cfg["H"], cfg["W"]
    row, col = beam_tables(H_, W_, cfg["el"][0], cfg["el"][1])
    # the scale rule uses the reference beam model of the named workload
    Href, Wref = WORKLOADS[name]["H"], WORKLOADS[name]["W"]
    d_az = 2.0 * math.pi / Wref
    d_el = math.radians(cfg["el"][1] - cfg["el"][0]) / max(Href - 1, 1)
    delta = max(d_az, d_el)
    scene = make_scene(cfg["kind"], K, cfg["n_boxes"])
    surf = sample_surfels(scene, cfg["n"], K, cfg["el"], delta, cfg["r_max"], cfg["origin_mode"],
                          blob_fraction=cfg.get("blob_fraction", 0.0), n_blobs=cfg.get("n_blobs", 0))
    prng = np.random.Generator(np.random.PCG64(100 + K))
    poses = []
    if cfg["pose"] == "identity":
        poses.append(make_pose(0.0, 0.0, 0.0))
    elif cfg["pose"] == "random":
        yaw = prng.uniform(0.0, 2.0 * np.pi)
        tx, ty = prng.uniform(-5.0, 5.0, size=2)
        poses.append(make_pose(yaw, tx, ty))
    elif cfg["pose"] == "trajectory":
        yaw0 = prng.uniform(0.0, 2.0 * np.pi)
        for f in range(cfg["n_poses"]):
            dist = 1.5 * f - 1.5 * (cfg["n_poses"] - 1) / 2
            yaw = yaw0 + math.radians(prng.normal(0.0, 2.0))
            poses.append(make_pose(yaw, dist * math.cos(yaw0), dist * math.sin(yaw0)))
    out = dict(name=name, H=H_, W=W_, row_sincos=row, col_sincos=col, scene=scene,
               poses=poses, pose=poses[0], delta=delta, **surf)
    if with_targets:
        tg = [targets_for_pose(scene, p, row, col, cfg["drop"], 200 + K) for p in poses]
        out["target_depth"] = tg[0][0]
        out["target_normal"] = tg[0][1]
        out["targets"] = tg
    return out
