"""Each pin set must catch plausible slips in the oracle.

Every case below compiles a copy of the oracle source with one deliberate
mistake (a dropped factor, a flipped sign, a swapped axis, a reversed
order...) into a temporary library, runs the oracle pin suite against it in
a subprocess, and requires that suite to fail.  Nothing here touches a GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "splotch_oracle.c")

MUTATIONS = {
    "half_exponent": ("double g = exp(-q2);", "double g = exp(-0.5 * q2);"),
    "drop_rho0": ("double tau = e->rho0 * column(st, q2);", "double tau = column(st, q2);"),
    "drop_phi": ("*I = *I * ex + E * tau * phi(xx);", "*I = *I * ex + E * tau;"),
    "front_to_back_painter": ("for (int64_t a = nlist - 1; a >= 0; --a) {",
                              "for (int64_t a = 0; a < nlist; ++a) {"),
    "swap_screen_axes": ("double u = xc * s + 0.5 * (double)c->W;\n    double v = yc * s + 0.5 * (double)c->H;",
                         "double u = yc * s + 0.5 * (double)c->W;\n    double v = xc * s + 0.5 * (double)c->H;"),
    "flip_x": ("double u = xc * s + 0.5 * (double)c->W;", "double u = -xc * s + 0.5 * (double)c->W;"),
    "sigma_not_scaled_by_depth": ("double sig = ((double)h * soh) * s;",
                                  "double sig = ((double)h * soh) * (c->persp ? c->focal : s);"),
    "pixel_corner_not_centre": ("double dx = ((double)i + 0.5) - e->p.u;", "double dx = ((double)i) - e->p.u;"),
    "bbox_off_by_half": ("double a = (u - r) - 0.5, b = (u + r) - 0.5;", "double a = (u - r), b = (u + r);"),
    "palette_no_interp": ("double w = p - (double)k;", "double w = 0.0;"),
    "absorb_uses_emission": ("A[c] = st->mode[s] == 1 ? (double)st->absorb[s] * ca[c] : 0.0;",
                             "A[c] = st->mode[s] == 1 ? (double)st->bright[s] * ca[c] : 0.0;"),
    "no_log_scale": ("gv = log10((double)value);\n        g0 = log10((double)vmin);\n        g1 = log10((double)vmax);",
                     "gv = value;\n        g0 = vmin;\n        g1 = vmax;"),
    "depth_cull_inclusive_near": ("if (!(zc > c->znear && zc <= c->zfar)) {", "if (!(zc > c->znear - 1e9 && zc <= c->zfar)) {"),
    # 3-D truncation of the density
    "trunc3d_no_erf": ("g *= erf(sqrt(rem > 0.0 ? rem : 0.0));", "g *= 1.0;"),
    "trunc3d_erf_of_f": ("g *= erf(sqrt(rem > 0.0 ? rem : 0.0));", "g *= erf(f);"),
    # emission read as a source function
    "source_reading_ignored": ("if (st->emission_is_source && st->mode[s] == 1) E[c] = A[c] * E[c];", ""),
    "source_reading_on_additive": ("if (st->emission_is_source && st->mode[s] == 1) E[c] = A[c] * E[c];",
                                   "if (st->emission_is_source) E[c] = A[c] * E[c];"),
    # general colouring
    "absorb_palette_ignored": ("if (st->pal_abs)\n", "if (0)\n"),
    "vector_swap_g_b": ("const float comp[3] = {P->value[k], P->value_g[k], P->value_b[k]};",
                        "const float comp[3] = {P->value[k], P->value_b[k], P->value_g[k]};"),
    "vector_range_first_component": ("            nc = 3;\n", "            nc = 1;\n"),
    # compensated summation
    "compensation_dropped": ("img[ch * np + (size_t)j * W + i] += cmp[ch * pc + (size_t)(j - ra) * W + i];",
                             "img[ch * np + (size_t)j * W + i] += 0.0 * cmp[ch * pc + (size_t)(j - ra) * W + i];"),
    "row_bands_reordered": ("paint_rows(st, v, list + cnt[b], cnt[b + 1] - cnt[b], W, H, ra, rb, img_out);",
                            "paint_rows(st, v, list + cnt[b], cnt[b + 1] - cnt[b] - (cnt[b + 1] > cnt[b]), W, H, ra, rb, img_out);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, SPLOTCH_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not detect mutation {name}:\n{r.stdout[-2000:]}"
