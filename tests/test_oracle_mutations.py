"""The oracle pins catch plausible mistakes.

Each case plants one slip in a temporary copy of the oracle source (on the CPU
only), rebuilds it and runs the pin suite against the copy, which must fail.
The slips cover every stage of the method: WENO coefficients and smoothness
indicators, the mirrored stencil, Lax-Friedrichs splitting, the flux difference
of Eq. (2), boundary maps, the Runge-Kutta coefficients and stage times, the
primitive recovery, the compensated totals and the analytic references, and
for the other schemes the FORCE flux, the MUSTA stages, the MUSCL slopes and
limiters, the local splitting speeds and the ideal-gas recovery.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("weno5 candidate", "q[1] = (-fm1 + 5.0 * f0 + 2.0 * fp1) / 6.0;",
     "q[1] = (-fm1 + 5.0 * f0 + 2.0 * fp1) / 5.9;"),
    ("mirrored stencil", "const int jm = c * len + (i + r - o) + G;       // mirrored",
     "const int jm = c * len + (i + r - o - 1) + G;       // mirrored"),
    ("adjoint mirrored stencil", "sm[o] = fm[c * len + (i + r - o) + G];\n",
     "sm[o] = fm[c * len + (i + r - o - 1) + G];\n"),
    ("flux difference sign",
     "L[c * ncell + id] += (Fh[c * (nd + 1) + i] - Fh[c * (nd + 1) + i + 1]) / g.h[d];",
     "L[c * ncell + id] += (Fh[c * (nd + 1) + i + 1] - Fh[c * (nd + 1) + i]) / g.h[d];"),
    ("rk3 stage-2 weights", "u2[q] = 0.75 * u[q] + 0.25 * (u1[q] + dt * L[q]);",
     "u2[q] = 0.7 * u[q] + 0.3 * (u1[q] + dt * L[q]);"),
    ("rk3 stage time", "apply_L(g, t + dt, u1.data(), L.data(), clamps);",
     "apply_L(g, t + 0.5 * dt, u1.data(), L.data(), clamps);"),
    ("weno5 beta", "b[1] = 13.0 / 12.0 * a1 * a1 + 0.25 * c1 * c1;",
     "b[1] = 13.0 / 11.0 * a1 * a1 + 0.25 * c1 * c1;"),
    ("lax-friedrichs sign", "sm[o] = 0.5 * (ff[jm] - uu[jm]);",
     "sm[o] = 0.5 * (uu[jm] - ff[jm]);"),
    ("outflow map", "c[d] = m < 0 ? 0 : nd - 1;", "c[d] = m < 0 ? 1 : nd - 1;"),
    ("weight exponent", "alpha[k] = d[k] / (g * g);", "alpha[k] = d[k] / g;"),
    ("primitive pressure", "p = (E * E - M2) / (E + D);", "p = (E * E - M2) / (E + 1.01 * D);"),
    ("weno7 beta", "+ 3129.0 / 80.0 * a3[k] * a3[k];", "+ 3129.0 / 81.0 * a3[k] * a3[k];"),
    ("weno7 beta stencil", "a1[1] = (5.0 * m2 - 27.0 * m1 + 15.0 * z0 + 7.0 * p1) / 24.0;",
     "a1[1] = (5.0 * m2 - 27.0 * m1 + 15.0 * z0 + 7.0 * p2) / 24.0;"),
    ("weno7 candidate", "q[2] = (-m1 + 7.0 * z0 + 7.0 * p1 - p2) / 12.0;",
     "q[2] = (-m1 + 7.0 * z0 + 7.0 * p1 - p2) / 12.1;"),
    ("weno7 linear weights",
     "const double D7[4] = {1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0};",
     "const double D7[4] = {1.0 / 35.0, 12.0 / 35.0, 17.0 / 35.0, 5.0 / 35.0};"),
    ("pressure in flux", "f[2] = u[2] * v[d] + (d == 1 ? p : T(0.0));",
     "f[2] = u[2] * v[d] + (d == 2 ? p : T(0.0));"),
    ("compensated sum", "c = (tt - s) - y;", "c = 0.0;"),
    ("hubble charge", "pr[4] = hub[2] * s * s * s;", "pr[4] = hub[2] * s * s;"),
    ("shock charge", "s.n_right_star = nR * ga * va / (gb * vb);",
     "s.n_right_star = nR * va / (gb * vb);"),
    ("adjoint weight sensitivity",
     "acc += omega[k] * F.Q[k][j] - 2.0 * omega[k] * (q[k] - fhat) / (eps + b[k]) * dbeta;",
     "acc += omega[k] * F.Q[k][j] - 1.0 * omega[k] * (q[k] - fhat) / (eps + b[k]) * dbeta;"),
    ("adjoint split", "double acc = 0.5 * (ap[q * len + mm + G] - am[q * len + mm + G]);",
     "double acc = 0.5 * (ap[q * len + mm + G] + am[q * len + mm + G]);"),
    ("adjoint face weight", "const double gi = (wr - wl) / g.h[d];", "const double gi = (wr + wl) / g.h[d];"),
    ("adjoint stage weight", "b1[q] = 0.25 * b2[q] + 0.25 * dt * tmp[q];",
     "b1[q] = 0.25 * b2[q] + 0.5 * dt * tmp[q];"),
    ("adjoint stage time", "vjp_L(*g, t + dt, u1.data(), b2.data(), tmp.data());",
     "vjp_L(*g, t + 0.5 * dt, u1.data(), b2.data(), tmp.data());"),
    # MUSTA-FORCE and MUSCL (Sec. 1.1)
    ("force centre weight", "F[c] = 0.25 * (fL[c] + 2.0 * fM[c] + fR[c])",
     "F[c] = 0.25 * (fL[c] + 1.0 * fM[c] + fR[c])"),
    ("force dissipation", "(uR[c] - uL[c]) / (4.0 * lam);", "(uR[c] - uL[c]) / (2.0 * lam);"),
    ("richtmyer state", "uM[c] = 0.5 * (uL[c] + uR[c]) - 0.5 * lam * (fR[c] - fL[c]);",
     "uM[c] = 0.5 * (uL[c] + uR[c]) - lam * (fR[c] - fL[c]);"),
    ("musta corrector sign", "uR[c] = uR[c] - lam * (fR[c] - F[c]);", "uR[c] = uR[c] + lam * (fR[c] - F[c]);"),
    ("musta stage count", "if (stage < g.musta_k) {", "if (stage < g.musta_k - 1) {"),
    ("muscl slope stencil", "double sj = limited_slope(g.limiter, s[2][c] - s[1][c], s[3][c] - s[2][c]);",
     "double sj = limited_slope(g.limiter, s[2][c] - s[1][c], s[3][c] - s[1][c]);"),
    ("muscl right state", "uR[c] = s[2][c] - 0.5 * sj;", "uR[c] = s[2][c] + 0.5 * sj;"),
    ("mc limiter", "0.5 * (aa + ab));", "1.0 * (aa + ab));"),
    ("van leer limiter", "return 2.0 * a * b / (a + b);", "return a * b / (a + b);"),
    ("superbee limiter", "return sg * std::max(std::min(2.0 * aa, ab), std::min(aa, 2.0 * ab));",
     "return sg * std::max(std::min(2.0 * aa, ab), std::min(aa, 1.5 * ab));"),
    ("musta face difference", "L[c * ncell + id] += (Fc[i] - Fc[i + 1]) / g.h[d];",
     "L[c * ncell + id] += (Fc[i] - Fc[i + 1]) / g.h[(d + 1) % 3];"),
    # local Lax-Friedrichs splitting and characteristic speeds
    ("local alpha stencil", "for (int o = 0; o < 2 * r; ++o) alpha = std::max(alpha, spd[(i - r + 1 + o) + G]);",
     "for (int o = 0; o < 2 * r; ++o) alpha = std::max(alpha, spd[(i - r + 2 + o) + G]);"),
    ("local split sign", "sm[o] = 0.5 * (ff[jm] - alpha * uu[jm]);", "sm[o] = 0.5 * (ff[jm] + alpha * uu[jm]);"),
    ("acoustic speed", "double disc = cs2 * (1.0 - v2) * (1.0 - v2 * cs2 - vd * vd * (1.0 - cs2));",
     "double disc = cs2 * (1.0 - v2) * (1.0 - v2 * cs2 - vd * vd * (1.0 + cs2));"),
    ("ideal sound speed", "return e + p > 0.0 ? g.gamma * p / (e + p) : 0.0;",
     "return e + p > 0.0 ? g.gamma * p / e : 0.0;"),
    # ideal-gas equation of state and its recovery
    ("ideal pressure", "double p = (gamma - 1.0) * (e - n);", "double p = (gamma - 1.0) * (e - 0.9 * n);"),
    ("ideal recovery charge", "double pm = ideal_pressure(g.gamma, E - M * mid, N * std::sqrt(1.0 - mid * mid));",
     "double pm = ideal_pressure(g.gamma, E - M * mid, N);"),
    ("ideal recovery energy", "e = E - M * speed;", "e = E - M * speed * speed;"),
    ("ideal prim2con", "u[4] = n * std::sqrt(W2);", "u[4] = n * W2;"),
    ("charge flux axis", "f[4] = u[4] * v[d];", "f[4] = u[4] * v[0];"),
]


def _run_mutant(base, idx, name, old, new, src):
    work = os.path.join(base, "m%02d" % idx)
    os.makedirs(os.path.join(work, "oracle"))
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), os.path.join(work, "oracle"))
    with open(os.path.join(work, "oracle", "rh_oracle.cpp"), "w") as f:
        f.write(src.replace(old, new, 1))   # the first occurrence
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(work, "tests"),
                    ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutations.py",
                                                  "test_gpu*", "test_zz*"))
    os.symlink(os.path.join(ROOT, "paper_1604_03360_amd"), os.path.join(work, "paper_1604_03360_amd"))
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-p", "no:xdist", "tests/test_oracle_pins.py",
                        "tests/test_oracle_pins_schemes.py"], cwd=work,
                       capture_output=True, text=True, timeout=600, env=env)
    return name, r.returncode, r.stdout[-1500:]


@pytest.mark.slow
def test_pins_catch_planted_mistakes(tmp_path):
    from concurrent.futures import ThreadPoolExecutor
    src = open(os.path.join(ROOT, "oracle", "rh_oracle.cpp")).read()
    for name, old, _ in MUTATIONS:
        assert src.count(old) >= 1, name
    with ThreadPoolExecutor(max_workers=4) as pool:
        futs = [pool.submit(_run_mutant, str(tmp_path), i, name, old, new, src)
                for i, (name, old, new) in enumerate(MUTATIONS)]
        results = [f.result() for f in futs]
    missed = [(name, out) for name, rc, out in results if rc == 0]
    assert not missed, "planted mistakes not caught: %s" % [m[0] for m in missed]
