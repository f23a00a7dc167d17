"""The oracle's pins must catch plausible mistakes. Each case plants one slip in
a copy of the oracle's C source (on the CPU), builds it, swaps it in, and checks
that at least one pin fails."""
import ctypes as C
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "cpapr_oracle.c")

# (name, original text, planted mistake, pins expected to notice)
MUTATIONS = [
    ("no-eps-clamp", "vals[k] / (mk > eps ? mk : eps)", "vals[k] / mk",
     ["test_phi_clamp_matches_dense", "test_phi_empty_rows_and_clamped_contribution"]),
    ("pi-drops-last-mode", "if (m == mode) continue;\n            const double* row = A[m] + (int64_t)idx[(int64_t)m * nnz + k] * R;\n            for (int r = 0; r < R; ++r) pi[r] *= row[r];",
     "if (m == mode || m == nmodes - 1) continue;\n            const double* row = A[m] + (int64_t)idx[(int64_t)m * nnz + k] * R;\n            for (int r = 0; r < R; ++r) pi[r] *= row[r];",
     ["test_phi_matches_dense_bruteforce", "test_phi_mass_identity"]),
    ("dot-wrong-row", "mk += B[i * R + r] * pi[r];", "mk += B[r] * pi[r];",
     ["test_phi_matches_dense_bruteforce", "test_phi_golden_hand_example"]),
    ("scatter-no-pi", "neumaier_add(&Phi[i * R + r], &comp[i * R + r], s * pi[r]);",
     "neumaier_add(&Phi[i * R + r], &comp[i * R + r], s);",
     ["test_phi_matches_dense_bruteforce", "test_phi_rank_one_closed_form"]),
    ("kkt-sign", "q = 1.0 - Phi[i * R + r];", "q = Phi[i * R + r] - 1.0;",
     ["test_mu_inner_kkt_break"]),
    ("mu-update-divides", "B[i * R + r] *= Phi_last[i * R + r];", "B[i * R + r] /= Phi_last[i * R + r];",
     ["test_mu_inner_n2_is_lee_seung_kl_nmf", "test_mu_inner_monotone_nonnegative_and_mass"]),
    ("shift-any-phi", "phi_prev[n][e] > 1.0", "phi_prev[n][e] >= 0.0",
     ["test_solve_inadmissible_zero_shift"]),
    ("shift-ignores-A", "if (An[e] < kappa_tol && phi_prev[n][e] > 1.0)", "if (phi_prev[n][e] > 1.0)",
     ["test_solve_inadmissible_zero_shift"]),
    ("lambda-not-updated", "lam[r] = s + c;", "(void)s; (void)c;",
     ["test_solve_rank_one_closed_form", "test_solve_mass_and_normalisation"]),
    ("loglik-drops-mass", "*out = (s + c) - mass;", "*out = (s + c);",
     ["test_loglik_matches_dense"]),
    ("mttkrp-no-value", "neumaier_add(&M[i * R + r], &comp[i * R + r], vals[k] * t[r]);",
     "neumaier_add(&M[i * R + r], &comp[i * R + r], t[r]);", ["test_mttkrp_matches_dense"]),
    ("pqnr-y-sign", "y[r] = g[r] - gprev[r];", "y[r] = gprev[r] - g[r];",
     ["pqnr:test_pqnr_converges_faster_than_mu"]),
    ("pqnr-armijo-sign", "if (df <= PQNR_SIGMA * gdel) accepted = 1;", "if (df >= PQNR_SIGMA * gdel) accepted = 1;",
     ["pqnr:test_pqnr_objective_decreases_every_step", "pqnr:test_pqnr_matches_independent_lbfgsb"]),
    ("pqnr-no-projection", "delta[r] = (nb > 0.0 ? nb : 0.0) - b[r];", "delta[r] = nb - b[r];",
     ["pqnr:test_pqnr_kkt_at_convergence", "pqnr:test_pqnr_matches_independent_lbfgsb"]),
    ("pqnr-decrease-drops-m", "term = log1p(dm / m);", "term = log1p(dm);",
     ["pqnr:test_pqnr_objective_decreases_every_step", "pqnr:test_pqnr_converges_faster_than_mu"]),
    ("pqnr-two-loop-sign", "if (fr[r]) q[r] += (a[c] - beta) * P.s[j][r];", "if (fr[r]) q[r] -= (a[c] - beta) * P.s[j][r];",
     ["pqnr:test_pqnr_converges_faster_than_mu", "pqnr:test_pqnr_matches_independent_lbfgsb"]),
    ("pqnr-five-trials", "#define PQNR_TRIALS 4", "#define PQNR_TRIALS 5",
     ["pqnr:test_pqnr_line_search_four_trials_then_mu_step"]),
    ("pqnr-three-trials", "#define PQNR_TRIALS 4", "#define PQNR_TRIALS 3",
     ["pqnr:test_pqnr_line_search_four_trials_then_mu_step"]),
    ("pqnr-fallback-keeps-pairs", "if (!accepted) P.count = 0;", "if (!accepted) (void)0;",
     ["pqnr:test_pqnr_line_search_four_trials_then_mu_step"]),
    ("pqnr-fallback-no-step", "for (int r = 0; r < R; ++r) delta[r] = -b[r] * g[r];",
     "for (int r = 0; r < R; ++r) delta[r] = 0.0;",
     ["pqnr:test_pqnr_line_search_four_trials_then_mu_step"]),
    ("pqnr-fallback-last-trial", "        if (!accepted) /* the MU step b .* phi, written as b + (-b .* g) */\n"
     "            for (int r = 0; r < R; ++r) delta[r] = -b[r] * g[r];\n", "",
     ["pqnr:test_pqnr_line_search_four_trials_then_mu_step"]),
    ("pdnr-hessian-drops-m", "const double w = sc / mm;", "const double w = sc;",
     ["pdnr:test_pdnr_first_step_is_damped_newton", "pdnr:test_pdnr_converges_in_few_steps"]),
    ("pdnr-hessian-no-cross-terms", "w * pi[r] * pi[c]", "w * pi[r] * pi[r]",
     ["pdnr:test_pdnr_first_step_is_damped_newton"]),
    ("pdnr-damping-unscaled", "trace += H[r * R + r];", "trace += 1.0;",
     ["pdnr:test_pdnr_first_step_is_damped_newton"]),
    ("pdnr-pivot-sign", "for (int k = 0; k < c; ++k) piv -= L[c * nf + k] * L[c * nf + k];",
     "for (int k = 0; k < c; ++k) piv += L[c * nf + k] * L[c * nf + k];",
     ["pdnr:test_pdnr_first_step_is_damped_newton"]),
    ("pdnr-backsolve-transposed", "v -= L[k * nf + a] * d[fidx[k]];", "v -= L[a * nf + k] * d[fidx[k]];",
     ["pdnr:test_pdnr_first_step_is_damped_newton"]),
    ("pdnr-damping-never-relaxed",
     "mu = mu / PDNR_MU_STEP > PDNR_MU_MIN ? mu / PDNR_MU_STEP : PDNR_MU_MIN;",
     "mu = mu * PDNR_MU_STEP < PDNR_MU_MAX ? mu * PDNR_MU_STEP : PDNR_MU_MAX;",
     ["pdnr:test_pdnr_converges_in_few_steps"]),
    ("pdnr-held-sign", "if (g[r] > 0.0 && b[r] <= PDNR_HELD) continue;", "if (g[r] < 0.0 && b[r] <= PDNR_HELD) continue;",
     ["pdnr:test_pdnr_converges_in_few_steps", "pdnr:test_pdnr_kkt_at_convergence"]),
]

PARAMS = {
    "test_phi_matches_dense_bruteforce": [((5, 4, 3), 3), ((3, 4, 2, 3), 2)],
    "test_mttkrp_matches_dense": [((5, 4, 3),)],
}


def _run_pin(name):
    if name.startswith("pqnr:"):
        from tests import test_oracle_pqnr as pq
        if name[5:] == "test_pqnr_line_search_four_trials_then_mu_step":
            for case in pq.CRAFTED:
                pq.test_pqnr_line_search_four_trials_then_mu_step(oracle, *case)
            return
        getattr(pq, name[5:])(oracle)
        return
    if name.startswith("pdnr:"):
        from tests import test_oracle_pdnr as pd
        getattr(pd, name[5:])(oracle)
        return
    fn = getattr(pins, name)
    cases = PARAMS.get(name, [()])
    for args in cases:
        fn(oracle, *args)


@pytest.mark.parametrize("name,orig,bad,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, monkeypatch, name, orig, bad, catchers):
    src = open(SRC).read()
    assert src.count(orig) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(orig, bad, 1)
    cfile = tmp_path / "mut.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(so), str(cfile), "-lm"])
    monkeypatch.setattr(oracle, "_lib", C.CDLL(str(so)))
    caught = []
    for pin in catchers:
        try:
            _run_pin(pin)
        except (AssertionError, RuntimeError, FloatingPointError, ValueError):
            caught.append(pin)
    assert caught, f"no pin noticed the planted mistake {name}"
