"""Mutation check of the oracle pins (CPU only; not collected by pytest).

Plants one plausible mistake at a time in a copy of oracle/lbm_oracle.c and
runs the oracle pin tests (test_oracle_maps.py, test_oracle_physics.py)
against each mutant; a good set of pins fails on every mistake that matters
in the studied regimes.  The committed oracle is never touched: every
mutant is built in its own directory under --workdir.

    python tests/mutation_check.py --workdir SCRATCH_DIR [name ...]

Prints, per mutant, the pins that fail; "none" is the unmutated copy and
must fail none.
"""
import argparse
import json
import os
import re
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUT = {
 "none": [],
 "marangoni_sign": [("+ (1.0 - s.nx * s.nx) * dsx - s.nx * s.ny * dsy", "- (1.0 - s.nx * s.nx) * dsx + s.nx * s.ny * dsy"),
                    ("+ (1.0 - s.ny * s.ny) * dsy - s.nx * s.ny * dsx", "- (1.0 - s.ny * s.ny) * dsy + s.nx * s.ny * dsx")],
 "delta_s_dropped": [("double delta_s = 1.5 * P->W * g2;", "double delta_s = g2;")],
 "theta_sign": [("s.theta = 4.0 * s.phi", "s.theta = -4.0 * s.phi")],
 "omega_T": [("s.w_T = 1.0 / (alpha / CS2 + 0.5);", "s.w_T = 1.0 / (alpha / CS2 + 1.0);")],
 "omega_nu": [("s.w_nu = 1.0 / (nu / CS2 + 0.5);", "s.w_nu = 1.0 / (nu / CS2 + 1.0);")],
 "abb_to_bounce_back": [("= -POP(post, 2, opposite(a), j, i) + 2.0 * WGT[a] * Tw;", "= POP(post, 2, opposite(a), j, i); (void)Tw;")],
 "pressure_correction_dropped": [("s.p = ps + 0.5 * (s.Fpx * s.ux + s.Fpy * s.uy);", "s.p = ps;")],
 "half_force_in_u_dropped": [("s.ux = (jx + 0.5 * CS2 * s.Ftx)", "s.ux = (jx)"), ("s.uy = (jy + 0.5 * CS2 * s.Fty)", "s.uy = (jy)")],
 "curvature_sign": [("double curv = dnx_dx + dny_dy;", "double curv = -(dnx_dx + dny_dy);")],
 "pressure_force_sign": [("s.Fpx = -dvx;", "s.Fpx = dvx;"), ("s.Fpy = -dvy;", "s.Fpy = dvy;")],
 "g_forcing_factor": [("(1.0 - 0.5 * w_nu) * s2d", "s2d")],
 "g_forcing_factor_11": [("+ (1.0 - 0.5 * w) * s[r];", "+ (r == 5 ? 1.0 : 1.0 - 0.5 * w) * s[r];")],
 "f_wall_bounce_back": [("POP(post, 0, mirror_y(a), j, is)", "POP(post, 0, opposite(a), j, i)")],
 "T_ghost_mirror": [("= 2.0 * T_bottom(P, i) - P1(w->T, 0, i);", "= P1(w->T, 0, i);"),
                    ("= 2.0 * P->T_c - P1(w->T, ny - 1, i);", "= P1(w->T, ny - 1, i);")],
 "stencil_scale": [("OUTX = sx_ / CS2;", "OUTX = sx_ / (2.0 * CS2);")],
 "sigma_TT_dropped": [("+ p->sigma_TT * d * d;", ";")],
 "mu_swap": [("double mu = interp(s.phi, P->mu_a, P->mu_b);", "double mu = interp(s.phi, P->mu_b, P->mu_a);")],
 "k_swap": [("double kc = interp(s.phi, P->k_a, P->k_b);", "double kc = interp(s.phi, P->k_b, P->k_a);")],
 "f_eq_second_order": [("M * theta * nyv, CS2 * phi, CS2 * phi,", "M * theta * nyv, 0.5 * phi, 0.5 * phi,")],
 "omega_phi": [("const double w_phi = 1.0 / (P->M_phi / CS2 + 0.5);", "const double w_phi = 1.0 / (P->M_phi / CS2 + 1.0);")],
 "h_eq_second_order": [("double ceq[9] = {T, 0.0, 0.0, CS2 * T, CS2 * T,", "double ceq[9] = {T, 0.0, 0.0, 0.5 * T, 0.5 * T,")],
 "g_force_scale": [("s[1] = CS2 * Ftx - ux * G;", "s[1] = Ftx - ux * G;"), ("s[2] = CS2 * Fty - uy * G;", "s[2] = Fty - uy * G;")],
 "g_eq_u2_dropped": [("eq[3] = p * CS2 + vphi * ux2;", "eq[3] = p * CS2;"), ("eq[4] = p * CS2 + vphi * uy2;", "eq[4] = p * CS2;")],
 "g_eq8_rho_dropped": [("eq[8] = CS2 * CS2 * CS2 * rho +", "eq[8] = CS2 * CS2 * CS2 +")],
 "gamma_sign": [("double G = Fpx * ux + Fpy * uy;", "double G = -(Fpx * ux + Fpy * uy);")],
 "theta_width": [("s.theta = 4.0 * s.phi * (1.0 - s.phi) / P->W;", "s.theta = 4.0 * s.phi * (1.0 - s.phi) / (2.0 * P->W);")],
 "wall_T_phase": [("return p->T_h + p->dT * cos(", "return p->T_h + p->dT * sin(")],
 "abb_weight": [("+ 2.0 * WGT[a] * Tw;", "+ WGT[a] * Tw;")],
 "x_stream_reversed": [("int js = j - EY[a], is = wrap(i - EX[a], nx);", "int js = j - EY[a], is = wrap(i + EX[a], nx);")],
 "u_without_cs2": [("s.ux = (jx + 0.5 * CS2 * s.Ftx) / (s.rho * CS2);", "s.ux = (jx + 0.5 * CS2 * s.Ftx) / (s.rho);")],
 "rho_interp_swapped": [("P1(w->rho, j, i) = interp(phi, P->rho_a, P->rho_b);", "P1(w->rho, j, i) = interp(phi, P->rho_b, P->rho_a);")],
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workdir", required=True, help="scratch directory for the mutant copies")
    ap.add_argument("names", nargs="*", help="mutants to run (default: all)")
    args = ap.parse_args()
    src = open(os.path.join(ROOT, "oracle", "lbm_oracle.c")).read()
    results = {}
    for name in args.names or list(MUT):
        d = os.path.join(os.path.abspath(args.workdir), name)
        shutil.rmtree(d, ignore_errors=True)
        os.makedirs(d)
        shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(d, "oracle"),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
        shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(d, "tests"),
                        ignore=shutil.ignore_patterns("__pycache__"))
        os.symlink(os.path.join(ROOT, "paper_2210_07501_amd"), os.path.join(d, "paper_2210_07501_amd"))
        s = src
        for a, b in MUT[name]:
            if s.count(a) != 1:
                raise SystemExit("mutant %s: pattern not found once: %r" % (name, a))
            s = s.replace(a, b)
        open(os.path.join(d, "oracle", "lbm_oracle.c"), "w").write(s)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                            "tests/test_oracle_maps.py", "tests/test_oracle_physics.py"],
                           cwd=d, capture_output=True, text=True)
        failed = sorted(set(re.findall(r"FAILED tests/\S+::(\S+)", r.stdout)))
        results[name] = failed
        print(name, "->", len(failed), "pins fail:", failed, flush=True)
    print(json.dumps({"caught": sum(1 for k, v in results.items() if k != "none" and v),
                      "mutants": sum(1 for k in results if k != "none")}))


if __name__ == "__main__":
    main()
