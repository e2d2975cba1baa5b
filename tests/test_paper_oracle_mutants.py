"""Planted mistakes in the reference of the paper's scheme (oracle/hj_paper.c):
each plausible mistake below (a sign, a dropped factor, a wrong index or
weight, a wrong comparison, a wrong boundary rule) is compiled into a copy of
the reference, and the CPU pins of tests/test_paper_pins.py must fail on
every copy.  This checks the pins, not the GPU: nothing here runs a kernel."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "hj_paper.c")

MUTANTS = [
 ("tanh derivative sign", "c1 = P->kappa / P->s * (1.0 - th * th);", "c1 = P->kappa / P->s * (1.0 + th * th);"),
 ("bump gradient sign", "(-2.0 * P->gam)", "(2.0 * P->gam)"),
 ("bump centre sign", "double dx = x[i] - sgn * P->mu[i];", "double dx = x[i] + sgn * P->mu[i];"),
 ("H uses c1 for block B", "P->s2 * c2 * block_norm(p, P->k, n);", "P->s2 * c1 * block_norm(p, P->k, n);"),
 ("H_p not normalised", "Hp[i] = nA > 0.0 ? P->s1 * c1 * p[i] / nA : 0.0;", "Hp[i] = nA > 0.0 ? P->s1 * c1 * p[i] : 0.0;"),
 ("H_x wrong block norm", "Hx[i] = P->s1 * nA * g1[i] + P->s2 * nB * g2[i];", "Hx[i] = P->s1 * nA * g1[i] + P->s2 * nA * g2[i];"),
 ("quadratic H_x drops dr/dx factor", "Hx[i] = (q * m1 + P->w) * x[i];", "Hx[i] = (0.5 * q * m1 + 0.5 * P->w) * x[i];"),
 ("Rosenbrock gradient sign", "- 400.0 * x[0] * b", "+ 400.0 * x[0] * b"),
 ("Rosenbrock weight", "100.0 * b * b", "10.0 * b * b"),
 ("field sign of H_p", "    for (int i = 0; i < n; ++i)\n        f[i] = -f[i];", "    (void)0;"),
 ("Lax integrand sign", "        v = s - H;", "        v = H - s;"),
 ("rectangle weight", "q += h * integrand(P, y);", "q += 0.5 * h * integrand(P, y);"),
 ("Euler direction", "yn[i] = y[i] + h * K1[i];", "yn[i] = y[i] - h * K1[i];"),
 ("Hopf <x,v> sign", "phi = gstar(P, end + n) + q - xv;", "phi = gstar(P, end + n) + q + xv;"),
 ("F2 takes the max", "if (gk < phi || (gk != gk && phi == phi)) {", "if (gk > phi || (gk != gk && phi == phi)) {"),
 ("alpha halving off by one", "if (++kM == O->M) {", "if (++kM > O->M) {"),
 ("stop after one small move", "else if (count == n)", "else if (count == 1)"),
 ("FD quotient halved", "double gj = (fp - phi) / O->fd_sigma;", "double gj = (fp - phi) / (2.0 * O->fd_sigma);"),
 ("momentum sign", "+ O->momentum * (v[j] - vp[j]);", "- O->momentum * (v[j] - vp[j]);"),
 ("Hopf value not negated", "out_u[b] = P->functional == HJP_HOPF ? -best : best;", "out_u[b] = best;"),
 ("certificate direction of grad g", "        unit(n, gg, u2);", "        memcpy(u2, gg, sizeof(double) * n);"),
 ("LF viscosity sign", "hjp_hamiltonian(P, pt, p) - 0.5 * ax * (pp - pm)", "hjp_hamiltonian(P, pt, p) + 0.5 * ax * (pp - pm)"),
 ("LF boundary extrapolation", "double l = i > 0 ? phi[(size_t)j * nx + i - 1] : 2.0 * c - phi[(size_t)j * nx + 1];", "double l = i > 0 ? phi[(size_t)j * nx + i - 1] : phi[(size_t)j * nx + 1];"),
 ("staggered Lax: no implicit solve for x", "            stagger_solve(P, xm, pl, 1, delta, xl);", "            (void)0;"),
 ("staggered Hopf: no implicit solve for p", "                stagger_solve(P, pm, xl, 0, delta, pl);", "                (void)0;"),
 ("staggered Lax: explicit p uses p_{n-1}", "                pl[i] = pm[i] + delta * Hx[i];", "                pl[i] = pm[i] - delta * Hx[i];"),
 ("staggered Hopf: g* at p_N", "        G -= gstar(P, Pm + n);", "        G -= gstar(P, Pm + (size_t)N * n);"),
 ("staggered Lax: certificate at p_0", "            Pm[i] += delta * Hx[i];", "            Pm[i] += 0.0 * Hx[i];"),
 ("staggered Hopf: H sum from 0", "        for (int m = 1; m <= N; ++m)\n            G -= delta", "        for (int m = 0; m <= N; ++m)\n            G -= delta"),
 ("staggered Hopf: correction sign", "                G += (Pm[(size_t)m * n + i] - Pm[(size_t)(m + 1) * n + i])", "                G += (Pm[(size_t)(m + 1) * n + i] - Pm[(size_t)m * n + i])"),
 ("staggered Lax: H at x_{n+1}", "            phi -= delta * hjp_hamiltonian(P, X + (size_t)m * n, Pm + (size_t)m * n);", "            phi -= delta * hjp_hamiltonian(P, X + (size_t)(m + 1) * n, Pm + (size_t)m * n);"),
 ("staggered Hopf: certificate at x_1", "        xc = X;\n        pc = Pm + n;", "        xc = X + n;\n        pc = Pm + n;"),
 ("RK4 stage weight", "q += h / 6.0 * (i1 + 2.0 * i2 + 2.0 * i3 + i4);", "q += h / 6.0 * (i1 + i2 + 2.0 * i3 + 2.0 * i4);"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    base = open(SRC).read()
    assert base.count(old) == 1, "the planted line is not in the reference any more"
    src = tmp_path / "mutant.c"
    src.write_text(base.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-I" + os.path.join(ROOT, "oracle"), "-o", str(so), str(src), "-lm"])
    env = dict(os.environ, HJ_PAPER_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_paper_pins.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"the pins missed the planted mistake: {name}\n{r.stdout[-2000:]}"
