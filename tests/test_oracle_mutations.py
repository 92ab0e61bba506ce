"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that the pin
suite rejects every one of them: a dropped term, a wrong sign, factor or index, a
transposed operand."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "gamma_exponent_sign": ("- xp - d->lgk - d->lth);", "- xp - d->lgk + d->lth);"),
    "gamma_dk_factor": ("d->dk_dm = 2 * m / s2;", "d->dk_dm = m / s2;"),
    "gamma_shape_transposed": ("d->k = m * m / s2;", "d->k = s2 / m;"),
    "quench_power": ("Q = 1 - 2 / y + 2 * L / (y * y);", "Q = 1 - 2 / y + 2 * L / y;"),
    "quench_deriv_sign": ("*dQ_dkB = dQdy * (-y / kB);", "*dQ_dkB = dQdy * (y / kB);"),
    "resolution_b_term": ("o->ds[3] = m / (2 * s);", "o->ds[3] = m / s;"),
    "resolution_c_dropped": ("ld s2 = a * a + b * m + c * c * m * m;", "ld s2 = a * a + b * m;"),
    "bin_width_dropped": ("*K = dx * dens_eval(d, xm, &a, &b);", "*K = dens_eval(d, xm, &a, &b);"),
    "bin_centre_edge": ("xb[j] = (M->reco_edges[j] + M->reco_edges[j + 1]) * 0.5;", "xb[j] = M->reco_edges[j];"),
    "gengamma_shape_power": ("k = m * m / (p * p * s2);", "k = m * m / (p * s2);"),
    "gengamma_scale_shift": ("lgammaq((__float128)k + (__float128)(1 / p))", "lgammaq((__float128)k + (__float128)p)"),
    "gengamma_scale_chain": ("d->dth_dm = d->th / m - d->th * dD * d->dk_dm;", "d->dth_dm = d->th / m;"),
    "spois_scale_transposed": ("d->g = s2 / m;", "d->g = m / s2;"),
    "spois_digamma_shift": ("(d->llam - digamma_l(t + 1))", "(d->llam - digamma_l(t))"),
    "emg_shift_sign": ("d->mug = m - d->tau;", "d->mug = m + d->tau;"),
    "emg_width_unreduced": ("d->sg = s * sqrtl(1 - shape * shape);", "d->sg = s;"),
    "emg_dsigma_sign": ("*rsg = sg / (t * t) * (r - ph) - y / (sg * t) * ph;",
                        "*rsg = sg / (t * t) * (r - ph) + y / (sg * t) * ph;"),
    "emg_cdf_tail_sign": ("*F = 0.5L * erfcl(-y / (sqrtl(2) * sg)) - t * r;", "*F = 0.5L * erfcl(-y / (sqrtl(2) * sg)) + t * r;"),
    "igam_series_deriv_sign": ("dS -= c * H;", "dS += c * H;"),
    "igam_cf_deriv": ("dan = i;", "dan = -i;"),
    "exact_bins_one_sided": ("*K = Fh < 0.5L ? Fh - Fl : Fcl - Fch;", "*K = Fh - Fl;"),
    "gauss_cdf_ds_sign": ("*ds = -z * r;", "*ds = z * r;"),
    "psd_not_renormalised": ("P[(size_t)s * K + k] = p[k] / Z;", "P[(size_t)s * K + k] = p[k];"),
    "psd_kappa_inverted": ("sg = mx[2 + 2 * c] * kappa;", "sg = mx[2 + 2 * c] / kappa;"),
    "psd_eta_sign": ("logl(w1 / (1 - w1)) + eta", "logl(w1 / (1 - w1)) - eta"),
    "empty_bin_term_dropped": ("*term = n > 0 ? mu - n * logl(mu) : mu;", "*term = n > 0 ? mu - n * logl(mu) : 0;"),
    "pull_factor": ("nll += 0.5L * z * z;", "nll += z * z;"),
    "rate_grad_no_exposure": ("gr[s] += g * eps * F[(size_t)j * S + s] * pk;", "gr[s] += g * F[(size_t)j * S + s] * pk;"),
    "window_off_by_one": ("for (int j = M->win_lo; j < M->win_hi && ok; j++)",
                          "for (int j = M->win_lo; j <= M->win_hi - 2 && ok; j++)"),
    "digamma_tail_sign": ("return r + logl(x) - 0.5L / x - tail;", "return r + logl(x) - 0.5L / x + tail;"),
    "line_at_grid_energy": ("E = (ld)M->line_energy[line_s];", "E = (ld)M->line_energy[line_s] + 0.5 * M->e_step;"),
    "tiny_mu_domain": ("if (n > 0 && !isfinite((double)n / (double)mu)) *range = 1;",
                       "if (n > 0 && !isfinite((double)n / (double)mu)) return 0;"),
    "discovery_sign": ("*t = 2.0 * (res_null->nll - res_free->nll);", "*t = 2.0 * (res_free->nll - res_null->nll);"),
    "discovery_signal_left_free": ("&& p != signal);", ");"),
    "mv_piece_sign": ("const ld sign = k0 < K ? -1 : 1;", "const ld sign = k0 < K ? 1 : -1;"),
    "mv_total_dropped": ("if (k0 == K || k == k0) n +=", "if (k == k0) n +="),
    "bfgs_update_sign": ("(rho * rho * yHy + rho) * sv[i] * sv[j]", "(rho * rho * yHy - rho) * sv[i] * sv[j]"),
}


def _run(name, tmp):
    a, b = MUTANTS.get(name, ("", ""))
    src = open(SRC).read()
    assert name == "control" or src.count(a) == 1, name
    d = os.path.join(tmp, name)
    os.makedirs(d)
    shutil.copy(os.path.join(ROOT, "oracle", "oracle.h"), d)
    with open(os.path.join(d, "oracle.c"), "w") as f:
        f.write(src.replace(a, b) if a else src)
    lib = os.path.join(d, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", lib, os.path.join(d, "oracle.c"),
                           "-lquadmath", "-lm"])
    env = dict(os.environ, GS_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_families.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return name, r.returncode


@pytest.mark.slow
def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(max_workers=6) as ex:
        res = list(ex.map(lambda n: _run(n, str(tmp_path)), ["control"] + sorted(MUTANTS)))
    assert res[0] == ("control", 0), "the unmutated copy must pass the pins"
    res = res[1:]
    survivors = [n for n, rc in res if rc == 0]
    assert not survivors, f"pins did not catch: {survivors}"
