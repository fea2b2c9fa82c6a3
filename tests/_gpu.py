"""GPU-test helpers: move a seeded workload to the device, run the renderer through its C
ABI, run the FP64 oracle on the same inputs and compare with the stated tolerances.

Tolerances (float32 renderer against the float64 oracle):
  depth, opacity  |x - x_ref| <= 1e-5 |x_ref|
  normal          max-abs component error <= 1e-4
  gradients       per surfel, max_c |g_c - g_ref,c| <= 1e-3 max(|g_ref|_2, 3e-2 mass), with |.|_2
                  the norm of the surfel's vector for that parameter (3 for means, 4 quats,
                  2 log-scales, 1 opacity logit) and mass the oracle's sum over rays of the
                  norms of the individual ray contributions.  A float32 sum can only be
                  accurate relative to the sum of the magnitudes of its terms; the floor
                  matters for gradients that nearly vanish by cancellation (coplanar
                  contributors render depth = t exactly, so moving one along the plane
                  changes nothing) and carry float32 noise of about eps32 x mass.
Tie rays -- a threshold decision within 1e-4 relative of its threshold, or two
consecutive contributors whose centre ranges differ by less than 2.4e-7 = 2^-22 relative
(the renderer's float32 range key is within about half an ulp of the range, so two keys can
only order two centres against their true order when the ranges are within two ulps),
where a float32 evaluation may legitimately decide differently -- are excluded from value
parity and reported; their upstream gradient is zeroed on both sides in gradient parity.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import ref

TIE_MARGIN = 1e-4
TIE_ORDER = 2.4e-7
SURF_KEYS = ("means", "quats", "log_scales", "opacity_logits")


def to_dev(w, device="cuda:0"):
    d = {k: torch.from_numpy(np.ascontiguousarray(w[k])).to(device) for k in SURF_KEYS}
    d["row_sincos"] = torch.from_numpy(np.ascontiguousarray(w["row_sincos"])).to(device)
    d["col_sincos"] = torch.from_numpy(np.ascontiguousarray(w["col_sincos"])).to(device)
    d["pose"] = torch.from_numpy(np.ascontiguousarray(w["pose"], dtype=np.float32))
    if "target_depth" in w:
        d["target_depth"] = torch.from_numpy(np.ascontiguousarray(w["target_depth"])).to(device)
        d["target_normal"] = torch.from_numpy(np.ascontiguousarray(w["target_normal"])).to(device)
    return d


def gpu_forward(ctx, dw, want_state=True, chunk=0):
    from paper_2607_04127_amd import lgsr
    S = {k: dw[k] for k in SURF_KEYS}
    return lgsr.lgsr_forward(ctx, S, dw["pose"], dw["row_sincos"], dw["col_sincos"], want_state=want_state,
                             opts=lgsr.default_opts(chunk=chunk))


def oracle_forward(w, ray_ids=None):
    return ref.forward(w, w["pose"], w["row_sincos"], w["col_sincos"], ray_ids=ray_ids, extra=True)


def tie_mask(of):
    return (of["margin"] < TIE_MARGIN) | (of["order_gap"] < TIE_ORDER)


def compare_forward(fr, of, ray_ids=None, rel=1e-5, natol=1e-4, conditioned=False):
    """Returns a dict of statistics; raises AssertionError on a parity failure.

    conditioned: the bars of a ray grow with 1 / den_min, the smallest |n'.d| among its
    contributors.  The renderer evaluates den = n'.d in float32 from the rounded normal (the
    ray direction enters exactly, as a float pair): |error| <= 3 * 2^-24 (half an ulp of each
    of the normal's three components, and the rounding of the sum).  t, u and v all carry den as a divisor,
    so q^2 = u^2 + v^2 moves by 2 q^2 |error| / den and G = exp(-q^2 / 2) by a relative
    q^2 |error| / den <= 9 * 1.8e-7 / den = 1.6e-6 / den.  The bars are therefore
    max(rel, 1.6e-6 / den_min) and max(natol, 1.6e-5 / den_min): unchanged for
    |n'.d| >= 0.16."""
    dep = fr["depth"].detach().cpu().numpy().reshape(-1).astype(np.float64)
    opa = fr["opacity"].detach().cpu().numpy().reshape(-1).astype(np.float64)
    nrm = fr["normal"].detach().cpu().numpy().reshape(-1, 3).astype(np.float64)
    drp = fr["drop"].detach().cpu().numpy().reshape(-1)
    if ray_ids is not None:
        dep, opa, nrm, drp = dep[ray_ids], opa[ray_ids], nrm[ray_ids], drp[ray_ids]
    tie = tie_mask(of)
    ok = ~tie
    hit = of["K"] > 0
    # rays with no hit in the oracle render exact zeros (ties aside)
    miss = ok & ~hit
    assert np.all(dep[miss] == 0) and np.all(opa[miss] == 0) and np.all(nrm[miss] == 0) and np.all(drp[miss] == 1), \
        "rays without a hit must render zeros"
    m = ok & hit
    e_d = np.abs(dep[m] - of["depth"][m]) / np.abs(of["depth"][m])
    e_a = np.abs(opa[m] - of["opacity"][m]) / np.abs(of["opacity"][m])
    e_n = np.abs(nrm[m] - of["normal"][m]).max(axis=1) if m.any() else np.zeros(0)
    stats = dict(rays=int(dep.shape[0]), hit=int(hit.sum()), tie=int(tie.sum()),
                 tie_threshold=int((of["margin"] < TIE_MARGIN).sum()), tie_order=int((of["order_gap"] < TIE_ORDER).sum()),
                 max_rel_depth=float(e_d.max(initial=0)), max_rel_opacity=float(e_a.max(initial=0)),
                 max_abs_normal=float(e_n.max(initial=0)))
    if conditioned:
        dmin = of["den_min"][m]
        rel = np.maximum(rel, 1.6e-6 / dmin)
        natol = np.maximum(natol, 1.6e-5 / dmin)
        stats.update(conditioned_rays=int((dmin < 0.16).sum()), min_den=float(dmin.min(initial=1.0)),
                     worst_of_bar=float(max((e_d / rel).max(initial=0), (e_a / rel).max(initial=0),
                                            (e_n / natol).max(initial=0))))
    bad_d, bad_a, bad_n = (e_d > rel).sum(), (e_a > rel).sum(), (e_n > natol).sum()
    assert bad_d == 0 and bad_a == 0 and bad_n == 0, (bad_d, bad_a, bad_n, stats)
    drop_ok = (drp[ok] == of["drop"][ok]) | (np.abs(of["opacity"][ok] - 0.5) < 1e-5)
    assert drop_ok.all(), ("drop mask", int((~drop_ok).sum()))
    return stats


def grad_check(g, g_ref, mass=None, rel=1e-3, floor=3e-2, per_row=True):
    """(failures, cosine, worst error / bound).  per_row: rows of a 2-D array are one
    surfel's vector; otherwise every element is checked on its own.  mass: per row (or per
    element) sum of contribution magnitudes; without it the floor is relative to the rms."""
    r = grad_report(g, g_ref, mass, rel, floor, per_row)
    return r["bad"], r["cos"], r["worst"]


def grad_report(g, g_ref, mass=None, rel=1e-3, floor=3e-2, per_row=True):
    """grad_check's outcome plus two diagnostics:
      floor_only -- rows within the bound only because of the mass floor (their error
                    exceeds rel * |g_ref row|);
      elem_bad   -- elements failing the plain element-wise rule
                    |g - g_ref| <= rel * max(|g_ref|, 1e-3 * rms(g_ref)),
      elem_bad_nonfloor -- of those, elements in rows that pass without the floor."""
    r = _grad_rows(g, g_ref, mass, rel, floor, per_row)
    g = np.asarray(g, np.float64).reshape(-1)
    gr = np.asarray(g_ref, np.float64).reshape(-1)
    rms = float(np.sqrt(np.mean(gr ** 2))) if gr.size else 0.0
    ebad = np.abs(g - gr) > rel * np.maximum(np.abs(gr), 1e-3 * rms) + 1e-30
    per = ebad.reshape(r["nrows"], -1).any(axis=1)
    r.update(elem_bad=int(ebad.sum()), elem_bad_rows=int(per.sum()),
             elem_bad_nonfloor=int((per & ~r["floor_rows"]).sum()), elems=int(gr.size))
    del r["floor_rows"]
    return r


def _grad_rows(g, g_ref, mass, rel, floor, per_row):
    g = np.asarray(g, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    if not per_row or g_ref.ndim == 1:
        g, g_ref = g.reshape(-1, 1), g_ref.reshape(-1, 1)
    if mass is None:
        scale = np.full(g_ref.shape[0], float(np.sqrt(np.mean(g_ref ** 2))) if g_ref.size else 0.0)
    else:
        scale = np.asarray(mass, np.float64).reshape(-1)
    err = np.abs(g - g_ref).max(axis=1)
    norm = np.linalg.norm(g_ref, axis=1)
    bound = rel * np.maximum(norm, floor * scale)
    bad = err > bound + 1e-30
    floor_rows = ~bad & (err > rel * norm + 1e-30)
    gf, rf = g.reshape(-1), g_ref.reshape(-1)
    cos = float(gf @ rf / (np.linalg.norm(gf) * np.linalg.norm(rf) + 1e-300))
    ratio = err / np.maximum(bound, 1e-300)
    w = int(np.argmax(ratio)) if ratio.size else -1
    worst_row = None if w < 0 else dict(row=w, g=g[w].tolist(), g_ref=g_ref[w].tolist(), scale=float(scale[w]),
                                        bound=float(bound[w]))
    return dict(bad=int(bad.sum()), cos=cos, worst=float(ratio.max(initial=0)),
                floor_only=int(floor_rows.sum()), rows=int(g_ref.shape[0]), nrows=int(g_ref.shape[0]),
                floor_rows=floor_rows, worst_row=worst_row, bad_rows=np.flatnonzero(bad)[:8].tolist())
