"""Plant plausible mistakes in a copy of the oracle and show the pins catch them.

Each mutation below edits one spot of a temporary copy of ``rt_oracle.c`` (a
dropped term, a wrong sign, a wrong index, a transposed operand, a swapped
coefficient), builds it with gcc, and runs the pin battery against that build
in a child process.  Every mutant must fail at least one pin; the unmutated
source must pass all of them.  Everything runs on the CPU.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rt_oracle.c")
BATTERY = os.path.join(ROOT, "tests", "oracle_battery.py")

# (name, old, new): `old` must occur in the source; its first occurrence is replaced.
# Not listed: flipping which sign of mu travels upward inside the operator is an
# equivalent mutant -- with a quadrature symmetric in mu the operator depends on
# |mu| only -- so no pin can (or should) reject it; the right-hand side, where the
# bottom inflow makes the direction observable, is mutated instead.
MUTATIONS = [
    ("t1_sign", "3.0 * mu * mu - 1.0", "3.0 * mu * mu + 1.0"),
    ("t2_sign", "*t2 = sqrt(2.0) * (3.0 * mu * mu - 3.0)", "*t2 = sqrt(2.0) * (3.0 - 3.0 * mu * mu)"),
    ("SI_uses_t2", "SI[k] = sig[2 * k] + t1 * sig[2 * k + 1];", "SI[k] = sig[2 * k] + t2 * sig[2 * k + 1];"),
    ("SQ_uses_t1", "SQ[k] = t2 * sig[2 * k + 1];", "SQ[k] = t1 * sig[2 * k + 1];"),
    ("J2_drops_Q", "sig[2 * k + 1] += w * (t1 * I[k] + t2 * Q[k]);", "sig[2 * k + 1] += w * (t1 * I[k]);"),
    ("J2_drops_I", "sig[2 * k + 1] += w * (t1 * I[k] + t2 * Q[k]);", "sig[2 * k + 1] += w * (t2 * Q[k]);"),
    ("weights_no_half", "0.5 * s->wmu[m]", "s->wmu[m]"),
    ("weights_no_phi", "(s->wnu[p] * s->phi[p] / norm)", "(s->wnu[p] / norm)"),
    ("J20_drops_xi", "sig[2 * k + 1] *= xi * s->W2;", "sig[2 * k + 1] *= s->W2;"),
    ("J20_drops_W2", "sig[2 * k + 1] *= xi * s->W2;", "sig[2 * k + 1] *= xi;"),
    ("apply_sign", "sout[i] = sin[i] - em[i];", "sout[i] = sin[i] + em[i];"),
    ("apply_wrong_output_index", "sout[i] = sin[i] - em[i];", "sout[i] = sin[i ^ 1] - em[i];"),
    ("series_pu_factor", "su += sgn * (double)(n - 1) * term;", "su += sgn * (double)n * term;"),
    ("series_sign", "double sgn = (n % 2 == 0) ? 1.0 : -1.0;", "double sgn = (n % 2 == 0) ? -1.0 : 1.0;"),
    ("closed_w1", "double w1 = w0 - d * e;", "double w1 = w0 - e;"),
    ("closed_pk", "*pk = w0 - *pu;", "*pk = 1.0 - *pu;"),
    ("swap_pu_pk_downward", "I[k] = E * I[u] + pu * S[u] + pk * S[k];",
     "I[k] = E * I[u] + pk * S[u] + pu * S[k];"),
    ("upwind_index", "int u = k - 1;", "int u = k + 1 < ns ? k + 1 : k - 1;"),
    ("kappa_times_mu", "double kappa = s->opac[p] / fabs(s->mu[m]);",
     "double kappa = s->opac[p] * fabs(s->mu[m]);"),
    ("kappa_drops_opacity", "double kappa = s->opac[p] / fabs(s->mu[m]);",
     "double kappa = 1.0 / fabs(s->mu[m]);"),
    ("trap_half_step", "double h = 0.5 * d;", "double h = d;"),
    ("euler_a", "*a = 1.0 / (1.0 + d);", "*a = 1.0 / (1.0 + 0.5 * d);"),
    ("euler_uses_upwind_source", "I[k] = a * I[u] + b * S[k];", "I[k] = a * I[u] + b * S[u];"),
    ("trap_beta", "*b = h / (1.0 + h);", "*b = h / (1.0 - h);"),
    ("rhs_drops_thermal", "b[2 * k] = b[2 * k] + s->eps * s->B[k];", "b[2 * k] = b[2 * k];"),
    ("rhs_inflow_wrong_side", "(with_t && upward) ? s->Ibot : 0.0", "(with_t && !upward) ? s->Ibot : 0.0"),
    ("rhs_Q_gets_inflow", "s->fs, SQ, 0.0,", "s->fs, SQ, inflow,"),
    ("diag_wrong_index", "d[j] = col[i];", "d[j] = col[j];"),
    ("gmres_mgs_sign", "for (l = 0; l < n; l++) w[l] -= h * V[(size_t)i * n + l];",
     "for (l = 0; l < n; l++) w[l] += h * V[(size_t)i * n + l];"),
    ("gmres_rotation_sign", "H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];",
     "H[(i + 1) * m + j] = sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];"),
    ("gmres_backsolve_transposed", "sum -= H[i * m + l] * y[l];", "sum -= H[l * m + i] * y[l];"),
    ("gmres_update_unpreconditioned", "precond(n, pc, w, z);\n        for (i = 0; i < n; i++) x[i] += z[i];",
     "precond(n, pc, w, z);\n        for (i = 0; i < n; i++) x[i] += w[i];"),
    ("gmres_left_bnorm_unpreconditioned", "bnorm = nrm2(n, z);", "bnorm = nrm2(n, b);"),
    ("gmres_left_true_residual_restart",
     "if (left) { precond(n, pc, r, z); memcpy(r, z, sizeof(double) * n); }\n        beta",
     "if (0) { precond(n, pc, r, z); memcpy(r, z, sizeof(double) * n); }\n        beta"),
    ("gmres_left_update_preconditioned", "if (left) memcpy(z, w, sizeof(double) * n);",
     "if (left) precond(n, pc, w, z);"),
    ("sor_transposed_triangle", "for (j = i + 1; j < n; j++) sum -= A[(size_t)i * n + j] * z[j];",
     "for (j = i + 1; j < n; j++) sum -= A[(size_t)j * n + i] * z[j];"),
    ("sor_drops_omega", "z[i] = sum / (A[(size_t)i * n + i] / om);", "z[i] = sum / A[(size_t)i * n + i];"),
    ("ssor_drops_D", "for (i = 0; i < n; i++) z[i] = A[(size_t)i * n + i] * z[i];", ""),
    ("ssor_scale_inverted", "z[i] = z[i] * ((2.0 - om) / om);", "z[i] = z[i] * (om / (2.0 - om));"),
    ("ssor_forward_uses_upper", "for (j = 0; j < i; j++) sum -= A[(size_t)i * n + j] * z[j];",
     "for (j = 0; j < i; j++) sum -= A[(size_t)j * n + i] * z[j];"),
    ("parab_pd_sign", "*pd = (w[2] - d * w[1])", "*pd = (d * w[1] - w[2])"),
    ("parab_pu_uses_d", "*pu = (w[2] + dd * w[1])", "*pu = (w[2] + d * w[1])"),
    ("parab_moment_series", "/ (double)(m + n + 1);", "/ (double)(m + n + 2);"),
    ("parab_downwind_index", "pd * S[k + 1]", "pd * S[k]"),
    ("parab_upward_downwind_step", "kappa * fabs(tau[k] - tau[k - 1])",
     "kappa * fabs(tau[k + 1] - tau[k])"),
    ("field_J_drops_xi", "        sig[2 * k] *= xi;\n", ""),
    ("field_rhs_no_inflow", "double inflow = (with_t && upward) ? s->Ibot : 0.0;",
     "double inflow = 0.0;"),
    ("field_apply_sign", "Iout[i] = Iin[i] - F[i];", "Iout[i] = Iin[i] + F[i];"),
    ("field_sigma_drops_c", "for (k = 0; k < s->ns; k++) sigma[2 * k] += s->eps * s->B[k];", ""),
    ("bicgstab_beta", "beta = (rho / rho_old) * (alpha / omega);", "beta = (rho / rho_old) * (omega / alpha);"),
    ("bicgstab_omega", "omega = dot(n, t, sv) / tt;", "omega = dot(n, sv, sv) / tt;"),
    ("bicgstab_x_update", "x[i] += alpha * ph[i] + omega * sh[i];", "x[i] += alpha * p[i] + omega * sh[i];"),
    ("cgs_p_update", "p[i] = u[i] + beta * (q[i] + beta * p[i]);", "p[i] = u[i] + beta * (q[i] + p[i]);"),
    ("cgs_q_sign", "q[i] = u[i] - alpha * v[i];", "q[i] = u[i] + alpha * v[i];"),
    ("cgs_x_unpreconditioned", "for (i = 0; i < n; i++) x[i] += alpha * uh[i];", "for (i = 0; i < n; i++) x[i] += alpha * uq[i];"),
    ("richardson_sign", "for (i = 0; i < n; i++) x[i] += z[i];\n    }", "for (i = 0; i < n; i++) x[i] -= z[i];\n    }"),
]


def _run_battery(lib_path):
    env = dict(os.environ, RT_ORACLE_LIB=lib_path)
    r = subprocess.run([sys.executable, BATTERY], env=env, capture_output=True, text=True,
                       timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-400:]


def _build(src_text, out_dir, name):
    c = os.path.join(out_dir, f"{name}.c")
    so = os.path.join(out_dir, f"lib{name}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", c,
                           "-o", so, "-lm"], stderr=subprocess.DEVNULL)
    return so


def _mutant(args):
    name, old, new, src, out_dir = args
    assert old in src, f"mutation {name}: pattern not found"
    so = _build(src.replace(old, new, 1), out_dir, name)
    rc, tail = _run_battery(so)
    return name, rc, tail


def test_unmutated_oracle_passes_battery(tmp_path):
    src = open(SRC).read()
    so = _build(src, str(tmp_path), "clean")
    rc, tail = _run_battery(so)
    assert rc == 0, tail


def test_every_planted_mistake_fails_a_pin():
    src = open(SRC).read()
    with tempfile.TemporaryDirectory() as d:
        jobs = [(n, o, w, src, d) for n, o, w in MUTATIONS]
        with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
            results = list(ex.map(_mutant, jobs))
    survivors = [(n, t) for n, rc, t in results if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
