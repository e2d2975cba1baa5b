"""Planted mistakes in the FP64 reference of the solver (oracle/hj_oracle.c):
each plausible mistake below (a sign, a dropped term or factor, a transposed
operand, a wrong stage offset or weight, a wrong comparison) is compiled into
a copy of the reference, and the CPU pins of tests/test_oracle_pins.py must
fail on every copy.  This checks the pins, not the GPU: nothing here runs a
kernel.  (old, new, k): the k-th occurrence of old is replaced."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "hj_oracle.c")

MUTANTS = [
    ("tanh c'' sign", "c2 = -2.0 * P->kappa / (P->s * P->s) * th * sech2;",
     "c2 = 2.0 * P->kappa / (P->s * P->s) * th * sech2;", 0),
    ("rational c' power", "c1 = P->kappa / (q * q);", "c1 = P->kappa / q;", 0),
    ("m'' of c^2 drops a term", "*m2 = 2.0 * c1 * c1 + 2.0 * c * c2;", "*m2 = 2.0 * c * c2;", 0),
    ("<Ax,p> transposed", "s += p[i] * P->A[i * P->n + j] * gam[j];",
     "s += p[i] * P->A[j * P->n + i] * gam[j];", 0),
    ("field: A^T p uses A", "Hx += P->A[j * n + i] * p[j];", "Hx += P->A[i * n + j] * p[j];", 0),
    ("field: H_x drops w", "double Hx = (q * m1 + P->w) * gam[i];",
     "double Hx = (q * m1) * gam[i];", 0),
    ("Hopf integrand sign", "val = H - xHx;", "val = xHx - H;", 0),
    ("Lax integrand sign of H", "val = pHp - H;", "val = pHp + H;", 0),
    ("g constant sign", "return 0.5 * s + P->j0;", "return 0.5 * s - P->j0;", 0),
    ("g* constant sign", "return 0.5 * s - P->j0;", "return 0.5 * s + P->j0;", 0),
    ("RK4 stage 3 offset", "Y[i] = y[i] + 0.5 * h * K2[i];", "Y[i] = y[i] + h * K2[i];", 0),
    ("RK4 weights", "ynext[i] = y[i] + h / 6.0 * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);",
     "ynext[i] = y[i] + h / 6.0 * (2.0 * K1[i] + K2[i] + 2.0 * K3[i] + K4[i]);", 0),
    ("trapezoid end weight", "acc += (k + 1 < N ? h : 0.5 * h) * hjo_integrand(P, y, y + n);",
     "acc += h * hjo_integrand(P, y, y + n);", 0),
    ("Hopf objective <x,v> sign", "phi = gstar_val(P, y + n) + acc - dot(n, x, v);",
     "phi = gstar_val(P, y + n) + acc + dot(n, x, v);", 0),
    ("vjp: m'' term sign", "+ 2.0 * q * m2 * gam_lp * gam[i];", "- 2.0 * q * m2 * gam_lp * gam[i];", 0),
    ("vjp: m' factor 2 dropped",
     "double mp = -m * P->d[i] * lg[i] + 2.0 * m1 * gam_lp * P->d[i] * p[i];",
     "double mp = -m * P->d[i] * lg[i] + m1 * gam_lp * P->d[i] * p[i];", 0),
    ("vjp: A^T lambda uses A", "mg -= P->A[j * n + i] * lg[j];", "mg -= P->A[i * n + j] * lg[j];", 0),
    ("integrand gradient (Hopf) drops m'", "cg = q * m1 - 2.0 * q * (m2 * r + m1) - P->w;",
     "cg = q * m1 - 2.0 * q * (m2 * r) - P->w;", 0),
    ("adjoint seed (Hopf) inverted", "lam[n + i] = P->a[i] * P->a[i] * yN[n + i];",
     "lam[n + i] = yN[n + i] / (P->a[i] * P->a[i]);", 0),
    ("adjoint stage offset index",
     "Kbar[i] = h / 6.0 * bw[s] * lam[i] + (s < 3 ? cst[s + 1] * h * Ybar[i] : 0.0);",
     "Kbar[i] = h / 6.0 * bw[s] * lam[i] + (s < 3 ? cst[s] * h * Ybar[i] : 0.0);", 0),
    ("tangent: dq term dropped",
     "double dHx = (dq * m1 + q * dm1) * gam[i] + (q * m1 + P->w) * dgam[i];",
     "double dHx = (q * dm1) * gam[i] + (q * m1 + P->w) * dgam[i];", 0),
    ("Lax certificate inverted", "res = yN[n + i] - yN[i] / (P->a[i] * P->a[i]);",
     "res = yN[n + i] - yN[i] * (P->a[i] * P->a[i]);", 0),
    ("Armijo term sign", "return trial <= cur - O->armijo_c * decrease + O->acc_rel * fabs(cur);",
     "return trial <= cur + O->armijo_c * decrease + O->acc_rel * fabs(cur);", 0),
    ("central difference halved", "double gj = (fp - fm) / (2.0 * O->fd_sigma);",
     "double gj = (fp - fm) / O->fd_sigma;", 0),
    ("Hopf value not negated", "out_u[b] = (P->formula == HJO_LAX) ? phi : -phi;",
     "out_u[b] = phi;", 0),
    ("ties go to the last slot",
     "|| (slot_cert[g] == pick_cert && slot_phi[g] < slot_phi[pick])) {",
     "|| (slot_cert[g] == pick_cert && slot_phi[g] <= slot_phi[pick])) {", 0),
    ("stop test inverted", "else if (smax < O->eps_step)", "else if (smax > O->eps_step)", 0),
    ("restarts go on after a certificate", "if (certified)\n                    break;",
     "if (0)\n                    break;", 0),
]


def _replace(text, old, new, k):
    pos = -1
    for _ in range(k + 1):
        pos = text.find(old, pos + 1)
        if pos < 0:
            return None
    return text[:pos] + new + text[pos + len(old):]


@pytest.mark.parametrize("name,old,new,k", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, k):
    mutated = _replace(open(SRC).read(), old, new, k)
    assert mutated is not None, "the planted line is not in the reference any more"
    src = tmp_path / "mutant.c"
    src.write_text(mutated)
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-I" + os.path.join(ROOT, "oracle"), "-o", str(so), str(src), "-lm"])
    env = dict(os.environ, HJ_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"the pins missed the planted mistake: {name}\n{r.stdout[-2000:]}"
