"""The pins catch planted mistakes in the oracle.

Each case compiles a copy of the oracle with one plausible mistake (a dropped
term, a wrong sign or index, a swapped constant, an off-by-one) into a
temporary library and runs the pin tests against it in a subprocess: at least
one pin must fail.  The oracle in the repository is never modified.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    # Moller-Trumbore: the third barycentric bound dropped
    "inside_without_u_plus_v": ("return u >= 0.0 && v >= 0.0 && u + v <= 1.0;", "return u >= 0.0 && v >= 0.0;",
                                "segment_triangle or worked_case or blocker"),
    # endpoint tolerance ignored at the start of a segment
    "eps_start_dropped": ("return inside_uv(u, v) && s > eps && s < L - eps;",
                          "return inside_uv(u, v) && s > 0.0 && s < L - eps;", "eps_end_interval"),
    # a multiplier constant of Philox changed in its last digit
    "philox_constant": ("M0 = 0xD2E7470EE14C6C93ull", "M0 = 0xD2E7470EE14C6C95ull", "philox"),
    # reflected energy uses the green albedo for every channel
    "albedo_channel": ("out[c] = (float)((double)e[c] * (double)rho[c]);",
                       "out[c] = (float)((double)e[c] * (double)rho[1]);", "energies or figure1 or gradient or coloured"),
    # origin update: wrong sign of the distance to the light plane
    "light_plane_sign": ("double sdist = dot3(q, n) / dn;", "double sdist = -dot3(q, n) / dn;", "light_update"),
    # Equation 2 tested on the green and blue channels only
    "eq2_channels_skipped": ("  for (int c = 0; c < 3; ++c) {\n    volatile float d = en[c] - eo[c];",
                             "  for (int c = 1; c < 3; ++c) {\n    volatile float d = en[c] - eo[c];", "equation2"),
    # Equation 2 made exclusive on the upper bound
    "eq2_exclusive": ("if (!(mte <= d && d <= te)) return 0;", "if (!(mte <= d && d < te)) return 0;", "eq2"),
    # Malley's lift with a dropped factor
    "cosine_lift": ("double z2 = (1.0 - ar) * (1.0 + ar);", "double z2 = (1.0 - ar);", "cosine or concentric"),
    # first invalid segment recorded one too late
    "start_off_by_one": ("out = info_make(cell, n, j, 1, 1);", "out = info_make(cell, n, j + 1, 1, 1);",
                         "worked_case or blocker or photon_on_moved"),
    # albedo gradient without the division by the albedo
    "gradient_term": ("g_albedo[3 * m + c] += ge / albedo[3 * m + c];", "g_albedo[3 * m + c] += ge;", "gradient"),
    # light sample along the wrong tangent
    "light_sample_axis": ("double a = (2.0 * u[0] - 1.0) * half[0], b = (2.0 * u[1] - 1.0) * half[1];\n"
                          "  for (int i = 0; i < 3; ++i) x0[i] = c[i] + a * eu[i] + b * ev[i];",
                          "double a = (2.0 * u[0] - 1.0) * half[0], b = (2.0 * u[1] - 1.0) * half[1];\n"
                          "  for (int i = 0; i < 3; ++i) x0[i] = c[i] + a * eu[i] + b * eu[i];", "light_sample"),
    # bounce sampled on the wrong side of the surface
    "normal_not_flipped": ("    if (dot3(n, w) > 0.0)\n      for (int i = 0; i < 3; ++i) n[i] = -n[i];",
                           "    if (dot3(n, w) < 0.0)\n      for (int i = 0; i < 3; ++i) n[i] = -n[i];",
                           "energies or initial_trace or retrace"),
    # the walk keeps the segment after a close re-hit without checking it
    "close_rehit_unchecked": ("          !hit_on_moved(s, vhit(st, p, j + 2)) &&\n"
                              "          !seg_blocked(c->A, xb, xc, s->band_trace, 0, amb)) {",
                              "          !hit_on_moved(s, vhit(st, p, j + 2))) {", "close_rehit"),
    # after an accepted far hit the next segment is only checked, not traced
    "far_hit_not_traced_on": ("      put_photon(st, p, j, hp, (uint32_t)h.tri, ej, s->radius);\n      ++j;\n      need = 1;",
                              "      put_photon(st, p, j, hp, (uint32_t)h.tri, ej, s->radius);\n      ++j;\n      need = 0;",
                              "far_hit"),
    # a re-sampled path keeps the reflected instead of the arriving energy at its new vertex
    "kept_vertex_energy": ("        put_photon(st, p, j, hp, (uint32_t)h.tri, ej, s->radius);\n        newn = naive_tail(",
                           "        put_photon(st, p, j, hp, (uint32_t)h.tri, en, s->radius);\n        newn = naive_tail(",
                           "energy_differs_after or figure1"),
    # equal-distance hits: the later triangle wins instead of the lowest id
    "tie_rule": ("if (tt < h.t || (tt == h.t && t < h.tri)) { h.t = tt; h.tri = t; }",
                 "if (tt <= h.t) { h.t = tt; h.tri = t; }", "tie"),
    # closest hit forgets the moved objects (re-traced rays pass through them)
    "closest_hit_skips_moved": ("    double tmax = h.tri >= 0 ? h.t : T_FAR;",
                                "    if (ch->obj != 0 && s->obj_moved[ch->obj]) continue;\n"
                                "    double tmax = h.tri >= 0 ? h.t : T_FAR;", "valid_at_new_frame"),
    # pre-reject chunk boxes built from the first vertex of each triangle only
    "chunk_box_one_vertex": ("      for (int v = 0; v < 3; ++v)\n        for (int k = 0; k < 3; ++k) {\n"
                             "          double x = s->verts[9 * t + 3 * v + k];",
                             "      for (int v = 0; v < 1; ++v)\n        for (int k = 0; k < 3; ++k) {\n"
                             "          double x = s->verts[9 * t + 3 * v + k];", "multi_chunk"),
    # the last triangle of every chunk skipped by the closest-hit search
    "closest_hit_chunk_tail": ("    for (int64_t t = ch->first; t < ch->first + ch->count; ++t) {\n"
                               "      double v[9], tt, u, vv;\n      tri_verts(s, t, v);\n      if (!mt_plane",
                               "    for (int64_t t = ch->first; t < ch->first + ch->count - 1; ++t) {\n"
                               "      double v[9], tt, u, vv;\n      tri_verts(s, t, v);\n      if (!mt_plane",
                               "multi_chunk or valid_at_new_frame"),
    # box test: the walk traces the first invalid segment even when only a box was reached
    "box_walk_always_traces": ("int j = (int)k, need = !(s->verify_boxes && !origin_moved);",
                               "int j = (int)k, need = 1;", "box_mode_walk"),
    # box test: a moved light's segment 0 is checked instead of traced
    "box_walk_ignores_moved_light": ("int origin_moved = k == 0 && l >= 0 && s->light_moved[l];",
                                     "int origin_moved = 0;", "box_mode_walk"),
    # a sampled bounce's photon placed along the incoming direction
    "tail_photon_direction": ("for (int i = 0; i < 3; ++i) xn[i] = x[i] + h.t * wn[i];",
                              "for (int i = 0; i < 3; ++i) xn[i] = x[i] + h.t * w[i];",
                              "photons_lie or valid_at_new_frame"),
    # Equation 1 with the kept share in place of the pruned share
    "dm_prune_share": ("const float prob = (float)(C - tgt) / (float)C;", "const float prob = (float)tgt / (float)C;",
                       "dm_prune"),
    # the fill spreads re-sampled paths by the targets instead of the deficits
    "dm_fill_targets": ("const int64_t def = tgt > have ? tgt - have : 0;", "const int64_t def = tgt;",
                        "dm_fill or dm_static"),
    # rings of equal radius steps instead of equal area
    "dm_ring_radius": ("const double fr = rho2 / s2 * nr;", "const double fr = rho / s2 * nr;",
                       "dm_cell or dm_cells"),
    # restricted sampling with the position cell's row and column swapped
    "dm_sample_swapped": ("const int64_t iv = pc % gv, iu = pc / gv;", "const int64_t iu = pc % gv, iv = pc / gv;",
                          "dm_restricted or dm_initial"),
    # a moved light's paths keep their old cells
    "dm_stale_cells": ("    if (s->light_moved[l]) {\n      double x0[3], x1[3], d[3];",
                       "    if (0) {\n      double x0[3], x1[3], d[3];", "dm_moving"),
    # a spot light's cone test inverted
    "spot_cone_inverted": ("    return z >= param[0];", "    return z <= param[0];", "spot"),
    # spot samples drawn over the whole hemisphere (disk not scaled to the cone)
    "spot_disk_unscaled": ("    l[0] *= sr;\n    l[1] *= sr;", "    l[0] *= 1.0;\n    l[1] *= 1.0;", "spot"),
    # a camera's field-of-view tangents swapped between u and v
    "camera_tangents_swapped": ("return fabs(a) <= param[0] && fabs(b) <= param[1];",
                                "return fabs(a) <= param[1] && fabs(b) <= param[0];", "camera"),
    # a camera's pixel index transposed
    "camera_cell_transposed": ("    return iu * dm[1] + iv;", "    return iv * dm[0] + iu;", "cells"),
    # restricted spot samples spread over the whole disk instead of the cone's
    "spot_restricted_radius": ("const double rho2 = ((double)ring + u[2]) / (double)nr * s2, rho = sqrt(rho2);",
                               "const double rho2 = ((double)ring + u[2]) / (double)nr, rho = sqrt(rho2);",
                               "uniform_over_cells"),
    # the cosine ratio of Equation 2's E_N inverted
    "cosine_ratio_inverted": ("const double ratio = co > 0.0 ? fabs(c2) / co : 0.0;",
                              "const double ratio = co > 0.0 ? co / fabs(c2) : 0.0;", "cosine_ratio"),
    # the old vertex's cosine taken along the new vertex's direction (ratio 1)
    "cosine_ratio_old_direction": ("        sub3(xc, xb, d3);", "        sub3(xc, hp, d3);", "cosine_ratio"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_detect_planted_mistake(name):
    old, new, select = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: %s" % name
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "oracle.c")
        open(c, "w").write(src.replace(old, new))
        open(os.path.join(d, "oracle.h"), "w").write(open(os.path.join(ROOT, "oracle", "oracle.h")).read())
        lib = os.path.join(d, "liboracle_mut.so")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-o", lib, c, "-lm"])
        env = dict(os.environ, PV_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", select],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 1, "mutation %s survived the pins:\n%s" % (name, r.stdout[-2000:])
