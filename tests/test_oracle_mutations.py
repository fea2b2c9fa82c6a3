"""The oracle's pins must catch plausible mistakes.  Each case plants one slip (a dropped
term, a wrong sign, a wrong index or scale, a transposed operand) in a temporary copy of
oracle/lgsr_ref.c, compiles the copy on the CPU and runs the pin tests against it in a
subprocess (LGSR_REF_LIB); at least one pin must fail.  The oracle itself is not touched."""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lgsr_ref.c")

# name -> (text in lgsr_ref.c, replacement)
MUTATIONS = {
    # forward
    "u_uses_minor_scale": ("e->u = dot3(s->a, e->delta) / s->s0;", "e->u = dot3(s->a, e->delta) / s->s1;"),
    "transmittance_half_step": ("T *= (1 - ahat);", "T *= (1 - 0.5 * ahat);"),
    "depth_weight_is_T": ("SD += w * t;", "SD += T * t;"),
    "normal_not_normalised": ("for (int c = 0; c < 3; ++c) normal[3 * i + c] = r.SN[c] / r.A;",
                              "for (int c = 0; c < 3; ++c) normal[3 * i + c] = r.SN[c];"),
    "orientation_flipped": ("s->sigma = dot3(s->n, s->mu) <= 0 ? 1.0 : -1.0;",
                            "s->sigma = dot3(s->n, s->mu) <= 0 ? -1.0 : 1.0;"),
    "order_ignores_range": ("if (ri < rj) return -1;\n    if (ri > rj) return 1;", "if (0) return -1;"),
    "quaternion_sign": ("a[1] = 2 * (x * y + w * z);", "a[1] = 2 * (x * y - w * z);"),
    "pose_transposed": ("o[j] = pose[j] * v[0] + pose[4 + j] * v[1] + pose[8 + j] * v[2];",
                        "o[j] = pose[4 * j] * v[0] + pose[4 * j + 1] * v[1] + pose[4 * j + 2] * v[2];"),
    "alpha_not_clamped": ("e->ahat = e->aG < p->alpha_max ? e->aG : p->alpha_max;", "e->ahat = e->aG;"),
    "faint_hits_kept": ("e->ok[3] = e->ahat >= p->alpha_thr;", "e->ok[3] = e->ahat >= 0;"),
    "no_early_stop": ("if (T < p->T_min) {\n            stopped = 1;", "if (0) {\n            stopped = 1;"),
    "gaussian_without_half": ("exp(-0.5 * e->q2)", "exp(-e->q2)"),
    "no_support_cutoff": ("double k2 = p->cutoff_sigma * p->cutoff_sigma;\n    e->den", "double k2 = INFINITY;\n    e->den"),
    "hits_behind_near_kept": ("e->ok[1] = e->t >= p->near;", "e->ok[1] = e->t >= 0;"),
    "depth_not_normalised": ("depth[i] = r.SD / r.A;", "depth[i] = r.SD;"),
    "drop_inverted": ("drop[i] = r.A < prm->drop_tau;", "drop[i] = r.A >= prm->drop_tau;"),
    # tie outputs (margin, order_gap) and the conditioning output den_min
    "margin_ignores_den_eps": ("e->gap[0] = rel_gap(fabs(e->den), p->den_eps);", "e->gap[0] = INFINITY;"),
    "margin_ignores_hit_near": ("e->gap[1] = rel_gap(e->t, p->near);", "e->gap[1] = INFINITY;"),
    "margin_ignores_cutoff": ("e->gap[2] = rel_gap(e->q2, k2);", "e->gap[2] = INFINITY;"),
    "margin_ignores_alpha_thr": ("e->gap[3] = rel_gap(e->aG, p->alpha_thr);", "e->gap[3] = INFINITY;"),
    "margin_ignores_alpha_max": ("margin = fmin(margin, rel_gap(e.aG, p->alpha_max));", "(void)0;"),
    "margin_ignores_T_min": ("if (want_extra) margin = fmin(margin, rel_gap(T, p->T_min));", "(void)0;"),
    "margin_ignores_centre_near": ("margin = fmin(margin, rel_gap(s->r, p->near));", "(void)0;"),
    "margin_ignores_cut_surfels": ("margin = fmin(margin, need);", "(void)0;"),
    "margin_cut_surfels_only_when_accepted": ("if (!accepted(&e)) need = fmax(need, flip_gap(&e));",
                                              "if (!accepted(&e)) need = INFINITY;"),
    "margin_rejected_surfel_smallest_gap": ("else if (!e->ok[k]) g = fmax(g, x);",
                                            "else if (!e->ok[k]) g = g == 0.0 ? x : fmin(g, x);"),
    "margin_every_gap_of_every_surfel": ("else if (!e->ok[k]) g = fmax(g, x);",
                                         "else g = g == 0.0 ? x : fmin(g, x);"),
    "margin_rejected_surfels_ignored": ("else if (!e->ok[k]) g = fmax(g, x);", "else g = INFINITY;"),
    "margin_absolute_gap": ("static double rel_gap(double x, double thr) { return fabs(x - thr) / fabs(thr); }",
                            "static double rel_gap(double x, double thr) { return fabs(x - thr); }"),
    "order_gap_to_first_contributor": ("        prev_r = s->r;\n", "        if (prev_r < 0) prev_r = s->r;\n"),
    "order_gap_absolute": ("order_gap = fmin(order_gap, rel_gap(s->r, prev_r));",
                           "order_gap = fmin(order_gap, fabs(s->r - prev_r));"),
    "den_min_signed": ("den_min = fmin(den_min, fabs(e.den));", "den_min = fmin(den_min, e.den);"),
    # loss
    "normal_loss_gradient_unprojected": (
        "for (int c = 0; c < 3; ++c) g_normal[3 * i + c] = f * (N[c] - cosv * Nh[c] / nn);",
        "for (int c = 0; c < 3; ++c) g_normal[3 * i + c] = f * N[c];"),
    "normal_term_over_depth_mask": ("cntN += mN;", "cntN += mD;"),
    "depth_term_over_all_rays": ("cntD += mD;", "cntD += 1;"),
    "depth_gradient_unmasked": ("if (g_depth) g_depth[i] = cntD > 0 ? w_depth * mD * sgn / cntD : 0.0;",
                                "if (g_depth) g_depth[i] = cntD > 0 ? w_depth * sgn / cntD : 0.0;"),
    "zero_normal_costs_nothing": ("sumN += mN * (nn > 0 ? 1.0 - dot3(Nh, N) / nn : 1.0);",
                                  "sumN += mN * (nn > 0 ? 1.0 - dot3(Nh, N) / nn : 0.0);"),
    # backward
    "backward_drops_later_hits": ("double d_ahat = h->T * cj - B / (1 - h->ahat);", "double d_ahat = h->T * cj;"),
    "clamp_passes_gradient": ("if (h->aG < prm->alpha_max) { d_alpha = d_ahat * h->G; d_G = d_ahat * s->alpha; }",
                              "{ d_alpha = d_ahat * h->G; d_G = d_ahat * s->alpha; }"),
    "opacity_gradient_without_mean_terms": (
        "double gbA = g_opacity[i] - (g_depth[i] * Dh + dot3(gN, Nh)) / A;", "double gbA = g_opacity[i];"),
    "later_sum_unweighted": ("B += w * cj;", "B += cj;"),
    "gaussian_gradient_sign": ("double d_q2 = -0.5 * h->G * d_G;", "double d_q2 = 0.5 * h->G * d_G;"),
    "footprint_gradient_unscaled": ("gDelta[c] = d_u * s->a[c] / s->s0 + d_v * s->b[c] / s->s1;",
                                    "gDelta[c] = d_u * s->a[c] + d_v * s->b[c];"),
    "range_gradient_misses_ray": ("double g_t = d_t + dot3(gDelta, d);", "double g_t = d_t;"),
    "centre_gradient_misses_plane": ("g_mu[c] = -gDelta[c] + g_t * s->n[c] / h->den;", "g_mu[c] = -gDelta[c];"),
    "v_gradient_uses_u": ("double d_u = 2 * h->u * d_q2, d_v = 2 * h->v * d_q2;",
                          "double d_u = 2 * h->u * d_q2, d_v = 2 * h->u * d_q2;"),
    "scale_gradient_sign": ("atomic_add(&g->s0, -d_u * h->u / s->s0);", "atomic_add(&g->s0, d_u * h->u / s->s0);"),
    "normal_gradient_sign": ("g_n[c] = -g_t * h->delta[c] / h->den + s->sigma * d_nt[c];",
                             "g_n[c] = g_t * h->delta[c] / h->den + s->sigma * d_nt[c];"),
    "quaternion_gradient_unprojected": (
        "for (int c = 0; c < 4; ++c) dq[c] = (dqh[c] - radial * s->qhat[c]) / s->qnorm;",
        "for (int c = 0; c < 4; ++c) dq[c] = dqh[c] / s->qnorm;"),
    "logit_gradient_missing_factor": ("*dlog = s->alpha * (1 - s->alpha) * g->alpha;\n    double c1[3]",
                                      "*dlog = s->alpha * g->alpha;\n    double c1[3]"),
    "log_scale_gradient_unscaled": ("s->qhat[c]) / s->qnorm;\n    dl[0] = s->s0 * g->s0;",
                                    "s->qhat[c]) / s->qnorm;\n    dl[0] = g->s0;"),
    "pose_translation_sign": ("dpose[c] = -g->mu[c];", "dpose[c] = g->mu[c];"),
    "quaternion_term_sign": ("Gb[0] * 2 * y - Gb[1] * 4 * x + Gb[2] * 2 * w", "Gb[0] * 2 * y - Gb[1] * 4 * x - Gb[2] * 2 * w"),
    "centre_gradient_not_rotated": ("sensor_to_world_dir(pose, g->mu, dm);",
                                    "for (int c = 0; c < 3; ++c) dm[c] = g->mu[c];"),
    "pose_rotation_misses_normal": ("cross3(s->n, g->n, c4);", "c4[0] = c4[1] = c4[2] = 0;"),
    "pose_rotation_sign": ("dpose[3 + c] = -(c1[c] + c2[c] + c3[c] + c4[c]);",
                           "dpose[3 + c] = (c1[c] + c2[c] + c3[c] + c4[c]);"),
    # full objective
    "surf_normal_seam_not_wrapped": ("nb->r = k * W + (j + 1) % W;", "nb->r = k * W + (j + 1 < W ? j + 1 : j);"),
    "surf_normal_one_sided": ("a[c] = depth[nb->r] * dr[c] - depth[nb->l] * dl[c];",
                              "a[c] = depth[nb->r] * dr[c] - depth[k * W + j] * dp[c];"),
    "surf_normal_not_turned": ("*sgn = vd > 0 ? -1.0 : 1.0;", "*sgn = 1.0;"),
    "surf_term_over_omega_s": ("double tNs = cntD > 0 ? lambda_n * lambda_ns * sumNs / cntD : 0.0;",
                               "double tNs = cntS > 0 ? lambda_n * lambda_ns * sumNs / cntS : 0.0;"),
    "bce_without_eps": ("sumA += log(opacity[i] + eps);", "sumA += log(opacity[i]);"),
    "stencil_row_sign": ("g_depth[nb.u] += dot3(du, gb);", "g_depth[nb.u] -= dot3(du, gb);"),
    "stencil_cross_transposed": ("cross3(b, gv, ga);", "cross3(gv, b, ga);"),
    "surf_gradient_unprojected": ("gv[c] = sgn * (gN[c] - gu * u[c]) / vn;", "gv[c] = sgn * gN[c] / vn;"),
    "bce_sign": ("double tA = cntD > 0 ? -lambda_alpha * sumA / cntD : 0.0;",
                 "double tA = cntD > 0 ? lambda_alpha * sumA / cntD : 0.0;"),
    "bce_gradient_without_eps": ("g_opacity[i] = -lambda_alpha / (cntD * (opacity[i] + eps));",
                                 "g_opacity[i] = -lambda_alpha / (cntD * opacity[i]);"),
    "surf_normal_unnormalised": ("double Ns[3] = {sgn * v[0] / vn, sgn * v[1] / vn, sgn * v[2] / vn};",
                                 "double Ns[3] = {sgn * v[0], sgn * v[1], sgn * v[2]};"),
    "scale_reg_squared": ("if (smax > s_max) sum += smax - s_max;",
                          "if (smax > s_max) sum += (smax - s_max) * (smax - s_max);"),
    "scale_reg_gradient_not_chained": ("g_log_scales[2 * i + k] = lambda_s * smax;",
                                       "g_log_scales[2 * i + k] = lambda_s;"),
    "scale_reg_first_axis_only": ("int k = sy > sx ? 1 : 0;", "int k = 0;"),
    # scan projection and target covariance
    "scan_rows_bottom_up": ("double f = (el_max - el) / step;", "double f = (el - el_min) / step;"),
    "scan_farthest_wins": ("if (index[pix] < 0 || r < depth[pix]) {", "if (index[pix] < 0 || r > depth[pix]) {"),
    "scan_seam_clamped": ("if (j < 0) j += W;", "if (j < 0) j = 0;"),
    "scan_normal_not_turned": ("double sgn = dot3(nv, p) > 0 ? -1.0 : 1.0;", "double sgn = 1.0;"),
    "scan_range_limits_ignored": ("if (!(r >= r_min && r <= r_max) || kf < 0 || kf > H - 1) continue;",
                                  "if (kf < 0 || kf > H - 1) continue;"),
    "scan_columns_truncated": ("double kf = floor(f + 0.5), jf = floor(g + 0.5);",
                               "double kf = floor(f + 0.5), jf = floor(g);"),
    "scan_elevation_over_range": ("double el = atan2(p[2], rxy);", "double el = atan2(p[2], r);"),
    "scan_ties_to_later_point": ("if (index[pix] < 0 || r < depth[pix]) {",
                                 "if (index[pix] < 0 || r <= depth[pix]) {"),
    "cov_eps_not_squared": ("eps * eps};", "eps};"),
    "cov_axes_transposed": (
        "S[r][c] = R[r][0] * d[0] * R[c][0] + R[r][1] * d[1] * R[c][1] + R[r][2] * d[2] * R[c][2];",
        "S[r][c] = R[0][r] * d[0] * R[0][c] + R[1][r] * d[1] * R[1][c] + R[2][r] * d[2] * R[2][c];"),
    "cov_scales_swapped": ("double d[3] = {exp(2 * log_scales[2 * i]), exp(2 * log_scales[2 * i + 1]), eps * eps};",
                           "double d[3] = {exp(2 * log_scales[2 * i + 1]), exp(2 * log_scales[2 * i]), eps * eps};"),
}


def _run_case(name, tmp):
    from oracle import build as oracle_build
    orig = open(SRC).read()
    a, b = MUTATIONS[name]
    src = os.path.join(tmp, f"{name}.c")
    with open(src, "w") as f:
        f.write(orig.replace(a, b, 1))
    # the copy includes its header from the oracle directory
    lib = oracle_build.build(src=src, out=os.path.join(tmp, f"lib_{name}.so"))
    env = dict(os.environ, LGSR_REF_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_tie_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_objective_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_scan_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-300:]


def test_mutations_apply():
    orig = open(SRC).read()
    for name, (a, _) in MUTATIONS.items():
        assert orig.count(a) == 1, f"{name}: the planted text must occur once in lgsr_ref.c"


def test_every_mutation_fails_a_pin(tmp_path):
    import shutil
    shutil.copy(os.path.join(ROOT, "oracle", "lgsr_ref.h"), tmp_path / "lgsr_ref.h")
    workers = min(8, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda n: _run_case(n, str(tmp_path)), MUTATIONS))
    survivors = [(n, last) for n, rc, last in results if rc == 0]
    for n, rc, last in results:
        print(f"{n:36s} rc={rc} {last}")
    assert not survivors, f"mutations that no pin caught: {survivors}"
