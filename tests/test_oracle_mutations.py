"""Plant plausible mistakes in a copy of the oracle source and check that
the pins in test_oracle.py, test_oracle_fsai.py, test_oracle_afsai.py,
test_oracle_interp.py, test_oracle_bamg.py and test_oracle_srqm.py catch
every one of them (CPU only)."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc.c")

# (name, exact text in orc.c, replacement)
MUTATIONS = [
    ("strength_strict", "-v[e] >= thr", "-v[e] > thr"),
    ("strength_count_transposed", "if (s) st_count[ci[e]] += 1;", "if (s) st_count[i] += 1;"),
    ("strength_sign", "double neg = -v[e];", "double neg = v[e];"),
    ("pmis_compare_flipped", "if (sym && key_greater(st_count, u, j, i)) sel = 0;",
     "if (sym && key_greater(st_count, u, i, j)) sel = 0;"),
    ("pmis_only_S", "int sym = strong[e] || (t >= 0 && strong[t]);", "int sym = strong[e]; (void)t;"),
    ("pmis_F_any_neighbour", "if (strong[e] && newc[ci[e]]) { next[i] = ORC_F; break; }",
     "if (newc[ci[e]]) { next[i] = ORC_F; break; }"),
    ("pmis_rand_low_bits", "return orc_splitmix64(seed, c) >> 11;", "return orc_splitmix64(seed, c) & ((1ull << 53) - 1);"),
    ("interp_no_lumping", "if (v[e] > 0.0) d = d + v[e];", "if (v[e] > 0.0) d = d;"),
    ("interp_sign", "pv[o] = -(alpha * v[e]) / d;", "pv[o] = (alpha * v[e]) / d;"),
    ("interp_alpha_inverted", "double alpha = num / den;", "double alpha = den / num;"),
    ("transpose_index", "ci[fill[c]] = i;", "ci[fill[c]] = c;"),
    ("spgemm_no_accumulate", "acc[j] = acc[j] + x * Y->val[t];", "acc[j] = x * Y->val[t];"),
    ("spgemm_wrong_operand", "acc[j] = acc[j] + x * Y->val[t];", "acc[j] = acc[j] + x * Y->val[e];"),
    ("chol_sign", "for (int32_t k = 0; k < j; ++k) t = t - a[(size_t)i * n + k] * a[(size_t)j * n + k];",
     "for (int32_t k = 0; k < j; ++k) t = t + a[(size_t)i * n + k] * a[(size_t)j * n + k];"),
    ("chol_solve_transposed", "for (int32_t k = i + 1; k < n; ++k) t = t - L[(size_t)k * n + i] * z[k];",
     "for (int32_t k = i + 1; k < n; ++k) t = t - L[(size_t)i * n + k] * z[k];"),
    ("omega_inverted", "return (4.0 / 3.0) / rho;", "return (4.0 / 3.0) * rho / 4.0;"),
    ("vcycle_restrict_wrong_vector", "spmv(&L->R, t, yc);", "spmv(&L->R, y, yc);"),
    ("vcycle_no_correction", "for (int32_t i = 0; i < n; ++i) s[i] = s[i] + t[i];",
     "for (int32_t i = 0; i < n; ++i) s[i] = s[i];"),
    ("vcycle_residual_sign", "for (int32_t i = 0; i < n; ++i) t[i] = y[i] - t[i];      /* r = y - A s */",
     "for (int32_t i = 0; i < n; ++i) t[i] = t[i] - y[i];"),
    ("pcg_beta_sign", "p[i] = z[i] + beta * p[i];", "p[i] = z[i] - beta * p[i];"),
    ("pcg_stop_nonstrict", "if (rtol > 0.0 && rn < rtol * bn) break;", "if (rtol > 0.0 && rn <= 10 * rtol * bn) break;"),
    ("fsai_no_scaling", "G->val[G->rp[i] + r] = g[r] / sd;", "G->val[G->rp[i] + r] = g[r];"),
    ("fsai_scale_not_sqrt", "double sd = sqrt(g[m - 1]);", "double sd = g[m - 1];"),
    ("fsai_wrong_unit_vector", "e[r] = r == m - 1 ? 1.0 : 0.0;", "e[r] = r == 0 ? 1.0 : 0.0;"),
    ("fsai_G_twice", "spmv(&L->G, y, u);\n        spmv(&L->GT, u, w);", "spmv(&L->G, y, u);\n        spmv(&L->G, u, w);"),
    ("fsai_omega_G_for_GT", "spmv(&GT, v, t);  /* t = G^T v */", "spmv(G, v, t);"),
    ("fsai_omega_quotient", "rq = vw / vv;", "rq = ww / vw;"),
    ("fsai_omega_fewer_steps", "for (int k = 0; k < ORC_FSAI_POWER_STEPS; ++k) {",
     "for (int k = 0; k < ORC_FSAI_POWER_STEPS - 5; ++k) {"),
    ("fsai_omega_pmis_seed", "orc_pmis_rand(seed + 1u, level, i)", "orc_pmis_rand(seed, level, i)"),
    ("fsai_step_sign", "s[i] = s[i] + L->omega * w[i];", "s[i] = s[i] - L->omega * w[i];"),
    ("ext_no_direct_coupling", "num[t] = e >= 0 ? v[e] : 0.0;", "num[t] = 0.0; (void)e;"),
    ("ext_no_sign_filter", "return sa == sd ? 0.0 : a;", "(void)sa; (void)sd; return a;"),
    ("ext_weak_in_set_lumped", "} else if (mark[k] != i) {", "} else if (!(strong[e] && cf[k] == ORC_C)) {"),
    ("ext_no_plus_i_diagonal", "if (plus_i) diag = diag + (v[e] * abar(rp, ci, v, k, i)) / D;", ";"),
    ("ext_denominator_without_i", "if (plus_i && set[ns - 1] < i) D = D + abar(rp, ci, v, k, i);", ";"),
    ("ext_union_takes_weak", "if (c != k && strong[f] && cf[c] == ORC_C && mark[c] != i)",
     "if (c != k && cf[c] == ORC_C && mark[c] != i)"),
    ("classical_fstar_dropped", "if (D == 0.0) { diag = diag + v[e]; continue; }", "if (D == 0.0) continue;"),
    ("ext_weight_sign", "pv[o + t] = -num[t] / diag;", "pv[o + t] = num[t] / diag;"),
    ("hybrid_tie_largest", "(deg == bestdeg && c < best)", "(deg == bestdeg && c > best)"),
    ("hybrid_degree_ignored", "for (int32_t b = 0; b < nf; ++b) deg += depends(rp, ci, strong, fp[b], c);",
     "deg = 1;"),
    ("hybrid_no_cover_update", "if (!depends(rp, ci, strong, fp[a], best)) fp[keep++] = fp[a];",
     "if (fp[a] != best) fp[keep++] = fp[a];"),
    ("bamg_tie_largest", "if (s > bn) { bn = s; best = t; }", "if (s >= bn && s > 0.0) { bn = s; best = t; }"),
    ("bamg_no_orthogonalization", "for (int32_t a = 0; a < nt; ++a) work[t * nt + a] = work[t * nt + a] - d * q[r][a];",
     "(void)d;"),
    ("bamg_back_substitution_sign", "for (int32_t k = m + 1; k < r; ++k) t = t - R[m][k] * w[k];",
     "for (int32_t k = m + 1; k < r; ++k) t = t + R[m][k] * w[k];"),
    ("bamg_never_adapts", "if (relres <= eps && wn <= mu && r > 0) break;", "break;"),
    ("bamg_residual_ignored", "*relres = ni > 0.0 ? sqrt(nr) / sqrt(ni) : 0.0;", "*relres = 0.0; (void)nr; (void)ni;"),
    ("bamg_weak_paths", "if (j == k || !strong[e] || mark[j] == i) continue;", "if (j == k || mark[j] == i) continue;"),
    ("bamg_orthonormalize_no_division", "x[a] = t / G[a * nt + a];", "x[a] = t;"),
    ("bamg_psmooth_sign", "val[o] = pv - s * av;", "val[o] = pv + s * av;"),
    ("bamg_psmooth_no_scaling", "double s = omega * dinv[i];", "double s = omega; (void)dinv;"),
    ("bamg_pfilter_keeps_smallest", "while (u >= 0 && (fabs(pv[ord[u]]) < fabs(pv[x]) ||",
     "while (u >= 0 && (fabs(pv[ord[u]]) > fabs(pv[x]) ||"),
    ("bamg_pfilter_no_compensation", "val[o] = pv[t] + d;", "val[o] = pv[t]; (void)d;"),
    ("bamg_pfilter_compensation_sign", "val[o] = pv[t] + d;", "val[o] = pv[t] - d;"),
    ("bamg_coarse_space_not_injected",
     "memmove(TV + (size_t)c * nt, TV + (size_t)i * nt, sizeof(double) * (size_t)nt);", "(void)i;"),
    ("srqm_residual_sign", "for (int32_t a = 0; a < nt; ++a) r = r - S[(size_t)i * m + a] * T[a * nt + b];",
     "for (int32_t a = 0; a < nt; ++a) r = r + S[(size_t)i * m + a] * T[a * nt + b];"),
    ("srqm_no_preconditioner", "S[(size_t)i * m + nt + b] = dinv[i] * R[(size_t)i * nt + b];",
     "S[(size_t)i * m + nt + b] = R[(size_t)i * nt + b];"),
    ("srqm_largest_ritz_values", "if (!used[k] && (best < 0 || lam[k] < lam[best])) best = k;",
     "if (!used[k] && (best < 0 || lam[k] > lam[best])) best = k;"),
    ("srqm_back_substitution_no_division", "Z[r * nt + b] = t / L[r * m + r];", "Z[r * nt + b] = t;"),
    ("srqm_gram_wrong_operand",
     "for (int32_t i = 0; i < n; ++i) h = h + S[(size_t)i * m + a] * AS[(size_t)i * m + b];",
     "for (int32_t i = 0; i < n; ++i) h = h + S[(size_t)i * m + a] * S[(size_t)i * m + b];"),
    ("srqm_keeps_dependent_columns", "if (!(d > 1e-12 * gmax)) continue;", "if (!(d > 0.0)) continue;"),
    ("srqm_symeig_rotation_sign", "const double s = t * c;", "const double s = -t * c;"),
    ("srqm_fsai_G_twice", "csr_block(GT, nt, Y, nt, S + nt, m);", "csr_block(G, nt, Y, nt, S + nt, m);"),
    ("fsai_jacobi_threshold_flipped", "lower_row_max(&L->A) <= ORC_FSAI_MAXROW", "lower_row_max(&L->A) > ORC_FSAI_MAXROW"),
    ("afsai_tie_largest", "(fabs(z[t]) == fabs(z[best]) && cand[t] < cand[best])",
     "(fabs(z[t]) == fabs(z[best]) && cand[t] > cand[best])"),
    ("afsai_signed_gradient", "fabs(z[t]) > fabs(z[best]) ||", "z[t] > z[best] ||"),
    ("afsai_candidates_in_pattern", "if (j < i && pos[j] < 0 && seen[j] != w->stamp)",
     "if (j < i && seen[j] != w->stamp)"),
    ("afsai_gradient_wrong_entry", "if (pos[c] >= 0) s = s + A->val[q] * y[pos[c]];",
     "if (pos[c] >= 0) s = s + A->val[q] * y[0];"),
    ("afsai_stop_inverted", "if (k > 0 && psi_prev - psi <= eps * psi_prev) break;",
     "if (k > 0 && psi_prev - psi > eps * psi_prev) break;"),
    ("afsai_psi_not_kept", "        psi_prev = psi;\n", "        (void)psi_prev;\n"),
    ("afsai_one_step_more", "if (k == steps) break;", "if (k == steps + 1) break;"),
    ("afsai_no_scaling", "for (int32_t r = 0; r < m; ++r) val[r] = y[r] / sd;",
     "for (int32_t r = 0; r < m; ++r) val[r] = y[r];"),
    ("afsai_fallback_flipped", "use_fsai = maxcand <= ORC_AFSAI_MAXCAND;", "use_fsai = maxcand > ORC_AFSAI_MAXCAND;"),
    ("fsai_jacobi_smoother_from_params", "int fsai = L->G.rp != NULL;  /* this level's smoother */",
     "int fsai = h->prm.smoother == ORC_SMOOTH_FSAI;"),
]


PIN_FILES = ["test_oracle.py", "test_oracle_fsai.py", "test_oracle_afsai.py", "test_oracle_interp.py",
             "test_oracle_bamg.py", "test_oracle_srqm.py"]


def _first_file(name):
    """The pin file that targets the mutated step runs first, so that with
    -x a caught mutation stops early; every pin file still runs."""
    if name.startswith("fsai"):
        return "test_oracle_fsai.py"
    if name.startswith("afsai"):
        return "test_oracle_afsai.py"
    if name.startswith(("ext_", "hybrid_", "classical_")):
        return "test_oracle_interp.py"
    if name.startswith("bamg_"):
        return "test_oracle_bamg.py"
    if name.startswith("srqm_"):
        return "test_oracle_srqm.py"
    return "test_oracle.py"


def _run_pins(libpath, name):
    env = dict(os.environ, CAMG_ORACLE_LIB=libpath, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1")
    first = _first_file(name)
    files = [first] + [f for f in PIN_FILES if f != first]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + [os.path.join(ROOT, "tests", f) for f in files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/found"
    mutated = src.replace(old, new)
    cfile = tmp_path / "orc.c"
    cfile.write_text(mutated)
    hdr = os.path.join(ROOT, "oracle")
    lib = tmp_path / "liborc_mut.so"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                           "-I", hdr, "-o", str(lib), str(cfile), "-lm"])
    assert _run_pins(str(lib), name) != 0, f"the pins did not catch mutation {name}"
