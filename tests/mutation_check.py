"""Plant plausible mistakes in a copy of the oracle and confirm that the CPU
pin tests catch every one of them.

Run:  python tests/mutation_check.py      (CPU only; a few minutes)

Each mutation edits one expression of oracle/oracle.c (every copy of it:
the all-core sweep repeats the global factor) in a temporary copy, builds
it, and runs the oracle pin tests against that build through
VCSGC_ORACLE_LIB.  A mutation that no test catches is reported and the
script exits non-zero.
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = [
    ("half pair energy dropped", "e[i] = or_embed(p, species[i], rho[i]) + 0.5 * ps;",
     "e[i] = or_embed(p, species[i], rho[i]) + ps;"),
    ("global factor sign", "xg = beta * kN * dnd * (dnd + 2.0 * tt);",
     "xg = beta * kN * dnd * (dnd - 2.0 * tt);"),
    ("global factor 2 dropped", "xg = beta * kN * dnd * (dnd + 2.0 * tt);",
     "xg = beta * kN * dnd * (dnd + tt);"),
    ("kappa not per site", "double kN = a->kappa / (double)n;", "double kN = a->kappa;"),
    ("neighbour embedding dropped", "  return own + pair + emb;", "  return own + pair;"),
    ("pair uses own species for j", "    int sj = species[nj[e]];\n    pair +=",
     "    int sj = species[i];\n    pair +="),
    ("rho commit sign", "if (any) rho[j] = rho[j] + delta;", "if (any) rho[j] = rho[j] - delta;"),
    ("local chemical term sign", "  double xl = beta * (du + dmu0 * (double)dn);\n  double lnu = log(u);",
     "  double xl = beta * (du - dmu0 * (double)dn);\n  double lnu = log(u);"),
    ("force density derivative swapped",
     "fp[i] * or_df(p, sj, r) + fp[j] * or_df(p, si, r)",
     "fp[i] * or_df(p, si, r) + fp[j] * or_df(p, sj, r)"),
    ("force direction", "double coef = s / r;", "double coef = -s / r;"),
    ("embedding derivative factor", "return rho > 0.0 ? -A / (2.0 * sqrt(rho)) : 0.0;",
     "return rho > 0.0 ? -A / sqrt(rho) : 0.0;"),
    ("philox key bump", "      k1 += PH_W1;", "      k1 += PH_W0;"),
    ("density uses own species", "s += or_f(p, species[nj[e]], nr[e]);", "s += or_f(p, species[i], nr[e]);"),
    ("neighbour cutoff inclusive of far pairs",
     "  if (r2 > 1.000001 * cutoff * cutoff) return 0;\n  double r = sqrt(r2);\n  if (r < cutoff) {",
     "  double r = sqrt(r2);\n  if (r < cutoff + 0.5) {"),
    ("site drawn from wrong word", "catoms[cstart[c] + (int64_t)or_index(t[0], (uint64_t)m)]",
     "catoms[cstart[c] + (int64_t)or_index(t[0], (uint64_t)m) / 2]"),
    ("local chain keeps rejected stages", "          else undo_all(&ulog, species, rho, vx, vy, vz);",
     "          else ulog.n = 0;"),
    ("local chain counts only the last step", "              nrec++;\n              dn_tot += dn;",
     "              nrec++;\n              dn_tot = dn;"),
    ("commit skips flip", "  species[i] = (uint8_t)s1;\n}", "  species[i] = (uint8_t)s;\n}"),
    ("delayed acceptance without the reverse-move factor",
     "double l2 = (-xl + (xr < 0.0 ? xr : 0.0)) - (-x1 < 0.0 ? -x1 : 0.0);",
     "double l2 = -xl - (-x1 < 0.0 ? -x1 : 0.0);"),
    ("flipped descriptor ignores the density shift", "      if (any) rj = rj + delta;\n    }\n    cnt[k]",
     "      (void)any;\n    }\n    cnt[k]"),
    ("MLP gradient skips the activation derivative", "      da2[k] = dh2 * or_dsilu(A.a2[k]);",
     "      da2[k] = dh2;"),
    ("thermostat friction sign", "*xi = *xi + q4 * ((2.0 * *K - g * kT) / Q);",
     "*xi = *xi - q4 * ((2.0 * *K - g * kT) / Q);"),
    ("thermostat velocity factor inverted", "double s = (1.0 - a) / (1.0 + a);",
     "double s = (1.0 + a) / (1.0 - a);"),
    ("kinetic energy without the half", "return 0.5 * or_tree_sum(n, work) / OR_ACC;",
     "return or_tree_sum(n, work) / OR_ACC;"),
    ("fixed-shape sum drops the last chunk", "int64_t nch = (n + 255) / 256;",
     "int64_t nch = n / 256;"),
    ("spline slopes one-sided everywhere",
     "double mk = k == 0 ? y[1] - y[0] : 0.5 * (y[k + 1] - y[k - 1]);",
     "double mk = y[k + 1] - y[k];"),
    ("spline derivative not scaled by the knot spacing",
     "if (der) *der = (((3.0 * a[3]) * t + 2.0 * a[2]) * t + a[1]) * inv_h;",
     "if (der) *der = (((3.0 * a[3]) * t + 2.0 * a[2]) * t + a[1]);"),
    ("tabulated pair function of the wrong species pair",
     "if (p->tab) return or_spline_eval(p->cphi[a + b], p->nr, r, p->inv_dr, NULL);",
     "if (p->tab) return or_spline_eval(p->cphi[a], p->nr, r, p->inv_dr, NULL);"),
    ("virial sign", "      acc += s * r;\n    }\n    w[i] = acc;", "      acc -= s * r;\n    }\n    w[i] = acc;"),
    ("barostat without the 3/g kinetic coupling", "c = exp(-(1.0 + 3.0 / g) * ve * (0.5 * h));",
     "c = exp(-ve * (0.5 * h));"),
    ("barostat momentum not thermostatted", "  *pe = *pe * s;\n", "\n"),
    ("external pressure with the wrong sign", "pe = pe + h * (3.0 * V * (P - p_ext)",
     "pe = pe + h * (3.0 * V * (P + p_ext)"),
    ("grown-domain weight m instead of 8 / m", "  *w = 8 / m;\n  return bits;", "  *w = m;\n  return bits;"),
    ("grown-domain high interval from the wrong end", "int lo = u < ld, hi = u >= e - ld;",
     "int lo = u < ld, hi = u >= ld;"),
    ("grown domains with eight times the stages",
     "              : grown     ? (((n + ncells - 1) / ncells) + K - 1) / K",
     "              : grown     ? 8 * ((((n + ncells - 1) / ncells) + K - 1) / K)"),
    ("relaxation step against the direction", "xt[i] = or_wrap(x[i] + a * dx[i], box[0]);",
     "xt[i] = or_wrap(x[i] - a * dx[i], box[0]);"),
    ("decrease test with the wrong sign", "if (Et <= E - CG_C1 * a * sl && Et < E) {",
     "if (Et <= E + CG_C1 * a * sl) {"),
    ("Polak-Ribiere terms swapped", "double b = (g_new - g_mix) / gg;",
     "double b = (g_mix - g_new) / gg;"),
    ("direction update keeps the old force", "dx[i] = gx[i] + b * dx[i];",
     "dx[i] = fx[i] + b * dx[i];"),
]

TESTS = ["tests/test_oracle_philox.py", "tests/test_oracle_eam.py",
         "tests/test_oracle_ensemble.py", "tests/test_oracle_md.py",
         "tests/test_oracle_surrogate.py", "tests/test_oracle_localchain.py",
         "tests/test_oracle_nvt.py", "tests/test_oracle_table.py", "tests/test_oracle_cg.py",
         "tests/test_oracle_npt.py", "tests/test_oracle_grown.py"]


def main():
    src = open(SRC).read()
    missed = []
    with tempfile.TemporaryDirectory() as td:
        for name, old, new in MUTATIONS:
            if src.count(old) < 1:
                print(f"[skip] {name}: pattern not found")
                missed.append(name)
                continue
            mut = os.path.join(td, "oracle.c")
            open(mut, "w").write(src.replace(old, new))
            lib = os.path.join(td, "liboracle_mut.so")
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                                   "-std=c11", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
                                   "-o", lib, mut, "-lm"])
            env = dict(os.environ, VCSGC_ORACLE_LIB=lib)
            r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                                *TESTS], cwd=ROOT, env=env, capture_output=True, text=True,
                               timeout=900)
            caught = r.returncode != 0
            print(f"[{'caught' if caught else 'MISSED'}] {name}")
            if not caught:
                missed.append(name)
    if missed:
        print("uncaught:", missed)
        sys.exit(1)
    print("all mutations caught")


if __name__ == "__main__":
    main()
