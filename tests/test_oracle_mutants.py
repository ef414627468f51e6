"""Mutation check of the oracle's pins (CPU only).

Each mutant plants one plausible mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, a swapped index or operand, a wrong rounding), is
built with gcc, and the whole pin suite (tests/test_oracle_pins.py) runs
against it in a child process.  The suite must fail for every mutant and pass
for the unmodified copy built the same way: a pin set that a mistake of this
kind survives would not be pinning the oracle.  The mistakes are planted in
temporary copies only; the oracle itself is never modified.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dart_oracle.c")

# name -> list of (exact text in the oracle, replacement); each text must occur once
MUTANTS = {
    # Eq. 14: Doppler factor
    "doppler_sign": [("double D = sqrt(1.0 - b2) / (1.0 + bs);",
                      "double D = sqrt(1.0 - b2) / (1.0 - bs);")],
    "doppler_no_lorentz": [("double D = sqrt(1.0 - b2) / (1.0 + bs);",
                            "double D = 1.0 / (1.0 + bs);")],
    "doppler_beta2_not_squared": [
        ("double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];",
         "double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2];")],
    # Eqs. 18-19: exponent
    "exponent_2_minus_alpha": [("double p = 2.0 + v->alpha;", "double p = 2.0 - v->alpha;")],
    "exponent_3_plus_alpha": [("double p = 2.0 + v->alpha;", "double p = 3.0 + v->alpha;")],
    # Eq. 2: retarded time
    "retarded_time_sign": [("v->t_obs - smid;\n    const orc_window *w = tl_win;",
                            "v->t_obs + smid;\n    const orc_window *w = tl_win;")],
    "retarded_time_at_entry": [("double ds = sb - sa;\n    double smid = 0.5 * (sa + sb);",
                                "double ds = sb - sa;\n    double smid = sa;")],
    # Eqs. 6-7: epoch weights
    "weights_swapped": [("m_out[0] = m;     w_out[0] = 1.0 - delta;",
                         "m_out[0] = m;     w_out[0] = delta;"),
                        ("m_out[1] = m + 1; w_out[1] = delta;",
                         "m_out[1] = m + 1; w_out[1] = 1.0 - delta;")],
    "weights_first_interval_width": [("double delta = (tbar - t[m]) / (t[m + 1] - t[m]);",
                                      "double delta = (tbar - t[m]) / (t[1] - t[0]);")],
    "no_temporal_window": [("if (!(tbar >= t[0] && tbar <= t[M - 1])) return 0;",
                            "if (0) return 0;")],
    "nearest_tie_to_later": [("m_out[0] = (dr < dl) ? m + 1 : m;",
                              "m_out[0] = (dr <= dl) ? m + 1 : m;")],
    "nearest_picks_floor": [("m_out[0] = (dr < dl) ? m + 1 : m;", "m_out[0] = m;")],
    # Eq. 19: the chord
    "chord_dropped": [("*acc += ds * sum;", "*acc += sum;")],
    "crossings_ignore_cell_size": [("double s = (k * g->cell[a] - o[a]) / d[a];",
                                    "double s = (k - o[a]) / d[a];")],
    # record addressing
    "cell_index_x_z_swapped": [("size_t c = ((size_t)iz * g->n[1] + iy) * g->n[0] + ix;",
                                "size_t c = ((size_t)ix * g->n[1] + iy) * g->n[2] + iz;")],
    "beta_x_y_swapped": [("double b[3] = {load_val(g->beta, g->dtype, 3 * r), "
                          "load_val(g->beta, g->dtype, 3 * r + 1),",
                          "double b[3] = {load_val(g->beta, g->dtype, 3 * r + 1), "
                          "load_val(g->beta, g->dtype, 3 * r),")],
    # camera
    "pixel_corner_not_centre": [("double u = (i + 0.5 - 0.5 * v->width) * v->pixel_scale;",
                                 "double u = (i - 0.5 * v->width) * v->pixel_scale;")],
    "ev_flipped": [("out12[6] = -ct * cp; out12[7] = -ct * sp; out12[8] = st;",
                    "out12[6] = ct * cp; out12[7] = ct * sp; out12[8] = -st;")],
    "eu_flipped": [("out12[3] = -sp; out12[4] = cp;", "out12[3] = sp; out12[4] = -cp;")],
    "nhat_sin_cos_phi_swapped": [("double nhat[3] = {st * cp, st * sp, ct};",
                                  "double nhat[3] = {st * sp, st * cp, ct};")],
    "centre_off_by_half_cell": [(": 0.5 * g->n[a] * g->cell[a];",
                                 ": 0.5 * (g->n[a] + 1) * g->cell[a];")],
    # exact temporal integration
    "exact_cut_sign": [("double s = v->t_obs - g->times[m];\n            if (s > s_in && s < s_out)",
                        "double s = v->t_obs + g->times[m];\n            if (s > s_in && s < s_out)")],
    "exact_counts_pieces": [("else if (r > 0 && lin != last_cell) {", "else if (r > 0) {")],
    # sub-domains (labelled mode)
    "placement_origin_sign": [("g->placed ? g->centre[a] - g->origin[a]",
                               "g->placed ? g->centre[a] + g->origin[a]")],
    "placement_ignores_centre": [("g->placed ? g->centre[a] - g->origin[a]",
                                  "g->placed ? 0.5 * g->n[a] * g->cell[a] - g->origin[a]")],
    # 16-bit decoding and round-on-read
    "bf16_decode_shift": [("uint32_t u = (uint32_t)((const uint16_t *)p)[idx] << 16;",
                           "uint32_t u = (uint32_t)((const uint16_t *)p)[idx] << 15;")],
    "f16_decode_bias": [("else v = ldexp(1.0 + fr / 1024.0, ex - 15);",
                         "else v = ldexp(1.0 + fr / 1024.0, ex - 14);")],
    "bf16_round_truncates": [("u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;",
                              "u = u & 0xffff0000u;")],
    "f16_round_truncates": [("double q = nearbyint(ldexp(x, -ulp_exp));",
                             "double q = trunc(ldexp(x, -ulp_exp));")],
    # snapshot-outer form
    "ring_slot_off_by_one": [("me = w->ring ? me % w->ne : me - w->e0;",
                              "me = w->ring ? (me + 1) % w->ne : me - w->e0;")],
}


def _build(src_text, out_dir, name):
    c = os.path.join(out_dir, f"orc_{name}.c")
    so = os.path.join(out_dir, f"liborc_{name}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared",
                           "-o", so, c, "-lm", "-lpthread"])
    return so


def _run_pins(lib):
    env = dict(os.environ, DART_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests",
                        "test_oracle_pins.py"), "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return r.returncode, (lines[0] if lines else r.stdout[-300:])


@pytest.fixture(scope="module")
def outcomes():
    src = open(SRC).read()
    jobs = {"unmodified": src}
    for name, edits in MUTANTS.items():
        text = src
        for old, new in edits:
            assert text.count(old) == 1, f"{name}: the text to mutate is no longer in the oracle: {old!r}"
            text = text.replace(old, new)
        jobs[name] = text
    with tempfile.TemporaryDirectory() as d:
        libs = {name: _build(text, d, name) for name, text in jobs.items()}
        with ThreadPoolExecutor(max_workers=4) as ex:
            res = dict(zip(libs, ex.map(_run_pins, libs.values())))
    return res


def test_unmodified_copy_passes_the_pins(outcomes):
    rc, msg = outcomes["unmodified"]
    assert rc == 0, msg


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(outcomes, name):
    rc, msg = outcomes[name]
    # 1: a test failed (2-5 would be an interrupted run or a collection error)
    assert rc == 1, f"mutant {name} survived the pins (exit {rc}): {msg}"
    print(f"{name}: {msg}")
