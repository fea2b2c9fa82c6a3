"""Pure-Python float64 restatement of the renderer for tiny inputs (<= a few dozen surfels and
rays).  TEST INFRASTRUCTURE ONLY.

It restates the same definition as lgsr_ref.c (arXiv 2607.04127, Sec. 3.1 map and
spherical projection, Sec. 3.4 rendered depth/opacity/normal) in the most literal form
possible, with Python floats and the ``math`` module, to cross-check the C oracle on
small cases.  Being a second transcription of one definition, it is a consistency check,
not an independent pin.
"""
from __future__ import annotations

import math


def _rot_columns(q):
    w, x, y, z = q
    a = (1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y))
    b = (2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x))
    n = (2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y))
    return a, b, n


def _dot(p, q):
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2]


def render(means, quats, log_scales, logits, pose, row_sincos, col_sincos, cutoff_sigma=3.0,
           alpha_thr=1 / 255, alpha_max=0.99, T_min=1e-4, near=0.2, den_eps=1e-6, drop_tau=0.5):
    """Returns a list over rays (row-major) of (depth, opacity, (nx, ny, nz), drop, K)."""
    P = [[float(pose[i][j]) for j in range(4)] for i in range(3)]

    def to_sensor(v):  # R^T v
        return tuple(sum(P[i][j] * v[i] for i in range(3)) for j in range(3))

    surf = []
    for i in range(len(means)):
        q = [float(c) for c in quats[i]]
        qn = math.sqrt(sum(c * c for c in q))
        if qn == 0:
            continue
        a, b, n = _rot_columns([c / qn for c in q])
        mu = to_sensor([float(means[i][c]) - P[c][3] for c in range(3)])
        a, b, n = to_sensor(a), to_sensor(b), to_sensor(n)
        r = math.sqrt(_dot(mu, mu))
        if r < near:
            continue
        sgn = 1.0 if _dot(n, mu) <= 0 else -1.0
        surf.append(dict(i=i, r=r, mu=mu, a=a, b=b, n=n, nt=tuple(sgn * c for c in n),
                         s0=math.exp(float(log_scales[i][0])), s1=math.exp(float(log_scales[i][1])),
                         alpha=1.0 / (1.0 + math.exp(-float(logits[i])))))
    surf.sort(key=lambda s: (s["r"], s["i"]))

    out = []
    for k in range(len(row_sincos)):
        sp, cp = float(row_sincos[k][0]), float(row_sincos[k][1])
        for j in range(len(col_sincos)):
            st, ct = float(col_sincos[j][0]), float(col_sincos[j][1])
            d = (cp * ct, cp * st, sp)
            T, A, SD, SN, K = 1.0, 0.0, 0.0, [0.0, 0.0, 0.0], 0
            for s in surf:
                den = _dot(s["n"], d)
                if abs(den) < den_eps:
                    continue
                t = _dot(s["n"], s["mu"]) / den
                if t < near:
                    continue
                hit = [t * d[c] - s["mu"][c] for c in range(3)]
                u = _dot(s["a"], hit) / s["s0"]
                v = _dot(s["b"], hit) / s["s1"]
                if u * u + v * v > cutoff_sigma ** 2:
                    continue
                ah = min(alpha_max, s["alpha"] * math.exp(-(u * u + v * v) / 2))
                if ah < alpha_thr:
                    continue
                w = T * ah
                A += w
                SD += w * t
                SN = [SN[c] + w * s["nt"][c] for c in range(3)]
                T *= 1 - ah
                K += 1
                if T < T_min:
                    break
            if K == 0:
                out.append((0.0, 0.0, (0.0, 0.0, 0.0), 1, 0))
            else:
                out.append((SD / A, A, tuple(c / A for c in SN), int(A < drop_tau), K))
    return out
