"""Mutation check of the oracle pins: each plausible mistake below (a wrong
sign, a swapped index, a dropped term, a transposed operand), planted in a
copy of the oracle source on the CPU, must make at least one pin of
tests/test_oracle_pins.py fail."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTANTS = {
    "hll_diffusion_sign": ("c1 * c2 / (c2 - c1) * (UR[k] - UL[k])",
                           "c1 * c2 / (c2 - c1) * (UL[k] - UR[k])"),
    "hll_wave_speed": ("T c2 = vmax(unL + cL, unR + cR);", "T c2 = vmax(unL + cL, unR - cR);"),
    "hll_tangential_operand": ("qL * utL}", "qL * unL}"),
    "hydrostatic_min": ("T zs = vmax(zm, zp);", "T zs = vmin(zm, zp);"),
    "drop_source_sL": ("f.sL = T(0.5 * g) * (hm * hm - hL * hL);", "f.sL = T(0.0);"),
    "centred_sign_x": ("T fcen = T(-g) *", "T fcen = T(g) *"),
    "modified_velocity_index": ("r.un_m = c.un - (r.h_p / c.h)", "r.un_m = c.un - (r.h_m / c.h)"),
    "z_deduction_index": ("r.z_m = eta_m - r.h_m;", "r.z_m = eta_m - r.h_p;"),
    "minmod_min_max": ("if (a >= T(0.0) && b >= T(0.0)) return vmin(a, b);",
                       "if (a >= T(0.0) && b >= T(0.0)) return vmax(a, b);"),
    "primitive_v_operand": ("v[k] = qy[k] / h[k];", "v[k] = qx[k] / h[k];"),
    "rate_y_tangential": ("pqx[s] = -(X1[s] / T(p.dx) + Y2[s] / T(p.dy));",
                          "pqx[s] = -(X1[s] / T(p.dx) + Y1[s] / T(p.dy));"),
    "wall_ghost_sign": ("qx[dst] = p.bc[0] == BC_WALL ? -qx[src] : qx[src];",
                        "qx[dst] = qx[src];"),
    "friction_h0_h1": ("qn / (h0 * h1);", "qn / (h0 * h0);"),
    "manning_exponent": ("(h1 * dcbrt(h1))", "(h1 * h1)"),
    "heun_average": ("T hn = T(0.5) * (h[s] + h2[s]);", "T hn = h2[s];"),
    "cfl_drop_y": ("double r = amax[0] / p.dx + amax[1] / p.dy;", "double r = amax[0] / p.dx;"),
    "green_ampt_sign": ("(T(psi) + h) / zf", "(T(psi) - h) / zf"),
    "rain_missing_dt": ("h = h + T(dt) * T(rate);", "h = h + T(rate);"),
    "first_order_reconstructs": ("    if (p.order == 1) return piecewise_constant(c);",
                                 "    if (p.order == 7) return piecewise_constant(c);"),
    "first_order_heun": ("    if (p.order == 1) {\n        for (size_t s = 0; s < n; ++s) {",
                         "    if (p.order == 7) {\n        for (size_t s = 0; s < n; ++s) {"),
    "rusanov_speed_sign": ("T c = vmax(dfabs(unL) + cL, dfabs(unR) + cR);",
                           "T c = vmax(dfabs(unL) - cL, dfabs(unR) + cR);"),
    "rusanov_full_diffusion": ("- T(0.5) * c * (UR[k] - UL[k]);", "- c * (UR[k] - UL[k]);"),
    "hyetograph_open_interval": ("if (p.rain_t[k] <= t) r = p.rain_r[k];",
                                 "if (p.rain_t[k] < t) r = p.rain_r[k];"),
    "hyetograph_next_value": ("if (p.rain_t[k] <= t) r = p.rain_r[k];",
                              "if (p.rain_t[k] <= t) r = p.rain_r[k + 1 < p.rain_n ? k + 1 : k];"),
    "rain_weight_ignored": ("const double rate = p.rain_w ? r * p.rain_w[s] : r;",
                            "const double rate = r;"),
    "ga_ks_field_ignored": ("const double ks = p.ks_f ? p.ks_f[s] : p.ks;",
                            "const double ks = p.ks;"),
    "ga_psi_field_ignored": ("const double psi = p.psi_f ? p.psi_f[s] : p.psi;",
                             "const double psi = p.psi;"),
    "ga_dtheta_field_ignored": ("const double dtheta = p.dtheta_f ? p.dtheta_f[s] : p.dtheta;",
                                "const double dtheta = p.dtheta;"),
    "kinetic_support_width": ("T s = dsqrt(T(1.5 * g) * h);", "T s = dsqrt(T(g) * h);"),
    "kinetic_right_side_bound": ("        a = vmin(a, T(0.0));", "        a = vmax(a, T(0.0));"),
    "kinetic_third_moment": ("/ (T(6.0) * s);", "/ (T(4.0) * s);"),
    "kinetic_tangential_side": ("F[2] = m0L * utL + m0R * utR;", "F[2] = m0L * utL + m0R * utL;"),
    "kinetic_cfl_speed": ("const double gs = flux == 2 ? 1.5 * g : g;", "const double gs = g;"),
    "imposed_outward_velocity_sign": ("T w = wet ? qo / hb : T(0.0);",
                                      "T w = wet ? -qo / hb : T(0.0);"),
    "imposed_h_invariant_dropped": ("T wg = (w + T(2.0) * c) - T(2.0) * dsqrt(T(g) * hg);",
                                    "T wg = w;"),
    "imposed_h_invariant_sign": ("T wg = (w + T(2.0) * c) - T(2.0) * dsqrt(T(g) * hg);",
                                 "T wg = (w - T(2.0) * c) + T(2.0) * dsqrt(T(g) * hg);"),
    "imposed_q_discharge_sign": ("        qog = -T(qb);", "        qog = T(qb);"),
    "imposed_q_invariant_term": ("return 2.0 * std::sqrt(g * x) - qb / x;",
                                 "return 2.0 * std::sqrt(g * x) + qb / x;"),
    "imposed_hq_discharge_sign": ("qog = -T(p.bc_q[side]);", "qog = T(p.bc_q[side]);"),
    "imposed_supercritical_test": ("if (w > c) {  // supercritical outflow: free",
                                   "if (w < -c) {  // supercritical outflow: free"),
    "imposed_side_signs": ("const double sg = (side == 0 || side == 2) ? -1.0 : 1.0;",
                           "const double sg = (side == 0 || side == 3) ? -1.0 : 1.0;"),
    "imposed_tangential_dropped": ("    qtg = hg * vt;", "    qtg = T(0.0);"),
    "rate_y_uses_dx": ("""        ph[s] = -(X0[s] / T(p.dx) + Y0[s] / T(p.dy));
        pqx[s] = -(X1[s] / T(p.dx) + Y2[s] / T(p.dy));
        pqy[s] = -(X2[s] / T(p.dx) + Y1[s] / T(p.dy));""",
                       """        ph[s] = -(X0[s] / T(p.dx) + Y0[s] / T(p.dx));
        pqx[s] = -(X1[s] / T(p.dx) + Y2[s] / T(p.dx));
        pqy[s] = -(X2[s] / T(p.dx) + Y1[s] / T(p.dx));"""),
    "infiltration_keeps_q": ("""        qx = qx * r;
        qy = qy * r;""", """        qx = qx * T(1.0);
        qy = qy * T(1.0);"""),
    "vfroe_dry_side_velocity": ("    if (!wetL) unL = unR;\n", "\n"),
    "vfroe_middle_depth_sign": ("T cs = vmax(ch + T(0.25) * (unL - unR), T(0.0));",
                                "T cs = vmax(ch + T(0.25) * (unR - unL), T(0.0));"),
    "vfroe_middle_velocity_sign": ("        u = uh + (cL - cR);", "        u = uh - (cL - cR);"),
    "vfroe_tangential_side": ("F[2] = q * (u >= T(0.0) ? utL : utR);",
                              "F[2] = q * (u >= T(0.0) ? utR : utL);"),
    "vfroe_left_branch": ("    if (uh - ch >= T(0.0)) {", "    if (uh + ch >= T(0.0)) {"),
    "eno_larger_slope": ("return dfabs(a) <= dfabs(b) ? a : b;", "return dfabs(a) >= dfabs(b) ? a : b;"),
    "eno_dry_cell_reconstructed": ("    if (!(c.h > T(h_eps))) {\n        r.h_m = r.h_p = c.h;",
                                   "    if (false) {\n        r.h_m = r.h_p = c.h;"),
    "modified_eno_cap": ("T cap = T(2.0) * c.h;", "T cap = T(4.0) * c.h;"),
    "imposed_ghost_not_wet_tested": ("const bool wet = hb > T(p.h_eps);", "const bool wet = true;"),
}


def build_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "swe_oracle.cpp")).read()
    assert src.count(old) >= 1, name
    path_src = os.path.join(tmp, f"{name}.cpp")
    with open(path_src, "w") as f:
        f.write(src.replace(old, new, 1))
    lib = os.path.join(tmp, f"lib_{name}.so")
    subprocess.check_call(["g++", *oracle.CFLAGS, path_src, "-o", lib])
    return lib


def run_pins(lib):
    """0 if every pin passes with the library `lib`; the quick pins run
    first and the slow ones only if the quick ones all pass."""
    env = dict(os.environ, SWE_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    for sel in ("not slow", "slow"):
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "-m", sel, os.path.join(HERE, "test_oracle_pins.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            return r.returncode
    return 0


def test_every_mutant_is_caught(tmp_path):
    names = sorted(MUTANTS)

    def one(name):
        return name, run_pins(build_mutant(name, str(tmp_path)))

    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        results = dict(ex.map(one, names))
    survivors = [n for n, rc in results.items() if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"


def test_unmutated_source_passes_the_same_run(tmp_path):
    src = os.path.join(ROOT, "oracle", "swe_oracle.cpp")
    lib = os.path.join(str(tmp_path), "lib_plain.so")
    subprocess.check_call(["g++", *oracle.CFLAGS, src, "-o", lib])
    assert run_pins(lib) == 0
