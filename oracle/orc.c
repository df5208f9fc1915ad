/*
 * Plain CPU FP64 oracle for classical-AMG-preconditioned CG.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library.  Written from
 * the paper "Chronos: a general purpose classical AMG solver for High
 * Performance Computing" (Isotton, Frigo, Spiezia, Janna; arXiv 2102.07417)
 * and the textbook definitions it cites.  Readings of passages the paper
 * leaves open are stated beside the code that takes them.
 *
 * Every loop runs in the plain index order written here; the file is built
 * with -ffp-contract=off so a*b+c is a rounded multiply then a rounded add.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

void orc_free(void *p) { free(p); }

void orc_csr_free(orc_csr *m) {
    if (!m) return;
    free(m->rp); free(m->ci); free(m->val);
    m->rp = NULL; m->ci = NULL; m->val = NULL;
    m->nrows = m->ncols = 0;
}

void orc_params_default(orc_params *p) {
    p->theta = 0.25;
    p->seed = 0;
    p->nu_pre = 1;
    p->nu_post = 1;
    p->omega = 0.0;
    p->max_levels = 25;
    p->max_coarse = 256;
    p->max_iter = 1000;
    p->smoother = ORC_SMOOTH_JACOBI;
    p->interp = ORC_INTERP_DIRECT;
    p->bamg_lmin = 1;
    p->bamg_lmax = 2;
    p->bamg_eps = 1e-3;
    p->bamg_mu = 10.0;
    p->psmooth = 0;
    p->pfilter = 1.0;
    p->srqm_iters = 0;
    p->afsai_steps = 10;
    p->afsai_step = 2;
    p->afsai_eps = 0.01;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Position of column j in row i, or -1 (rows are sorted). */
static int32_t find_in_row(const int32_t *rp, const int32_t *ci, int32_t i, int32_t j) {
    int32_t lo = rp[i], hi = rp[i + 1] - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (ci[mid] == j) return mid;
        if (ci[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Input check.  The paper's problem is A x = b with A sparse SPD
 * (Section 1, eq. linSys), stored in CSR (Section 3, CSRMAT).  Checks, in
 * this order: row pointer shape, column range and strict ordering, finite
 * values, diagonal present, structural and numerical symmetry
 * (|a_ij - a_ji| <= 1e-12 max|a|), positive diagonal.
 */
int orc_validate(int32_t n, const int32_t *rp, const int32_t *ci, const double *v) {
    if (n < 1 || !rp || !ci || !v) return ORC_E_ARG;
    if (rp[0] != 0) return ORC_E_CSR;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return ORC_E_CSR;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return ORC_E_CSR;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return ORC_E_CSR;
        }
    double amax = 0.0;
    for (int32_t e = 0; e < rp[n]; ++e) {
        if (!isfinite(v[e])) return ORC_E_CSR;
        if (fabs(v[e]) > amax) amax = fabs(v[e]);
    }
    for (int32_t i = 0; i < n; ++i)
        if (find_in_row(rp, ci, i, i) < 0) return ORC_E_CSR;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t j = ci[e];
            int32_t t = find_in_row(rp, ci, j, i);
            if (t < 0) return ORC_E_CSR;
            if (fabs(v[e] - v[t]) > 1e-12 * amax) return ORC_E_CSR;
        }
    for (int32_t i = 0; i < n; ++i)
        if (!(v[find_in_row(rp, ci, i, i)] > 0.0)) return ORC_E_NOT_SPD;
    return ORC_OK;
}

/*
 * Classical strength of connection (Section 2, Strength of Connection,
 * eq. cla) filtered by a threshold theta.  The printed formula is garbled
 * (its denominator is a minimum of raw entries and is negative for an
 * M-matrix); the reading taken is the Ruge-Stueben measure it stands for:
 *   m_i = max_{k != i} (-a_ik),
 *   j in S_i  <=>  j != i, m_i > 0 and -a_ij >= theta * m_i.
 * theta * m_i is one rounded product; the test is a comparison, not a
 * division.  A row with no negative off-diagonal has no strong connection.
 * strong[e] flags entry e of A (aligned with col_idx); st_count[j] = |S_j^T|,
 * the number of rows that depend strongly on j.
 */
void orc_strength(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                  double theta, uint8_t *strong, int32_t *st_count) {
    for (int32_t i = 0; i < n; ++i) st_count[i] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int have = 0;
        double m = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] == i) continue;
            double neg = -v[e];
            if (!have || neg > m) { m = neg; have = 1; }
        }
        double thr = theta * m;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            int s = 0;
            if (ci[e] != i && have && m > 0.0 && -v[e] >= thr) s = 1;
            strong[e] = (uint8_t)s;
            if (s) st_count[ci[e]] += 1;
        }
    }
}

/*
 * splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the generator's state advances by the golden
 * gamma 0x9E3779B97F4A7C15 per draw and each output is the state passed
 * through the variant-13 finaliser.  orc_splitmix64(seed, c) is draw number
 * c (from 0) of a generator seeded with `seed`.
 */
uint64_t orc_splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The random part of the PMIS measure of point i on level l: the top 53 bits
 * of draw ((l << 40) + i). */
uint64_t orc_pmis_rand(uint64_t seed, int32_t level, int32_t i) {
    uint64_t c = ((uint64_t)(uint32_t)level << 40) + (uint64_t)(uint32_t)i;
    return orc_splitmix64(seed, c) >> 11;
}

/* key(a) > key(b) for the PMIS measure (|S^T|, random, index) compared
 * lexicographically. */
static int key_greater(const int32_t *cnt, const uint64_t *u, int32_t a, int32_t b) {
    if (cnt[a] != cnt[b]) return cnt[a] > cnt[b];
    if (u[a] != u[b]) return u[a] > u[b];
    return a > b;
}

/*
 * PMIS coarsening (Section 2, Strength of Connection, last paragraph; the
 * algorithm is the one of De Sterck, Yang and Heys, which the paper cites
 * but does not print).  Measure of i: |S_i^T| plus a random number in
 * [0, 1); here the tuple (|S_i^T|, 53-bit random, i) compared as integers,
 * which orders points the same way with a deterministic tie break.
 *   - points with |S_i^T| = 0 start as F, the rest undecided (U);
 *   - each round, every undecided i whose measure beats that of every
 *     undecided j in S_i u S_i^T becomes C (all selections of a round are
 *     made against the round's starting state);
 *   - then every undecided point that depends strongly on a new C point
 *     becomes F;
 *   - rounds repeat until no point is undecided.
 * cf[i] is ORC_C or ORC_F on return.
 */
int orc_pmis(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
             const int32_t *st_count, uint64_t seed, int32_t level, int8_t *cf, int32_t *rounds) {
    uint64_t *u = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int8_t *newc = (int8_t *)malloc((size_t)n);
    int8_t *next = (int8_t *)malloc((size_t)n);
    if (!u || !newc || !next) { free(u); free(newc); free(next); return ORC_E_NOMEM; }
    int32_t und = 0;
    for (int32_t i = 0; i < n; ++i) {
        u[i] = orc_pmis_rand(seed, level, i);
        cf[i] = (st_count[i] == 0) ? ORC_F : ORC_U;
        if (cf[i] == ORC_U) ++und;
    }
    int32_t r = 0;
    while (und > 0) {
        ++r;
        for (int32_t i = 0; i < n; ++i) {
            newc[i] = 0;
            if (cf[i] != ORC_U) continue;
            int sel = 1;
            for (int32_t e = rp[i]; e < rp[i + 1] && sel; ++e) {
                int32_t j = ci[e];
                if (j == i || cf[j] != ORC_U) continue;
                int32_t t = find_in_row(rp, ci, j, i);
                int sym = strong[e] || (t >= 0 && strong[t]);
                if (sym && key_greater(st_count, u, j, i)) sel = 0;
            }
            newc[i] = (int8_t)sel;
        }
        for (int32_t i = 0; i < n; ++i) {
            next[i] = cf[i];
            if (cf[i] != ORC_U) continue;
            if (newc[i]) { next[i] = ORC_C; continue; }
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                if (strong[e] && newc[ci[e]]) { next[i] = ORC_F; break; }
        }
        und = 0;
        for (int32_t i = 0; i < n; ++i) {
            cf[i] = next[i];
            if (cf[i] == ORC_U) ++und;
        }
    }
    if (rounds) *rounds = r;
    free(u); free(newc); free(next);
    return ORC_OK;
}

/*
 * Direct (distance-one) interpolation, P = [W; I] in the paper's F/C block
 * form (Section 2, eq. prolOperator), kept in the original ordering
 * (the F/C reordering of eq. blk_FC is notational).  Coarse index of a C
 * point: the number of C points before it.
 *   C row i: a single 1 in column cmap(i).
 *   F row i, C_i^S = S_i n C (neighbour sets of Section 2, Interpolation):
 *     d_i     = a_ii + sum of the positive off-diagonals of row i
 *               (positive couplings are never strong, so they are lumped),
 *     alpha_i = (sum of the negative off-diagonals) / (sum_{j in C_i^S} a_ij),
 *     w_ij    = -(alpha_i a_ij) / d_i  for j in C_i^S.
 *   This is the direct formula of the multigrid literature the paper cites
 *   (Stueben; Trottenberg, Oosterlee, Schueller).  An F row with no strong
 *   C neighbour is empty.  Sums run in CSR order, d_i starting from a_ii.
 */
int orc_interp_direct(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                      const uint8_t *strong, const int8_t *cf, orc_csr *P) {
    int32_t *cmap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!cmap) return ORC_E_NOMEM;
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i) { cmap[i] = nc; if (cf[i] == ORC_C) ++nc; }
    int32_t *prp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!prp) { free(cmap); return ORC_E_NOMEM; }
    prp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = 0;
        if (cf[i] == ORC_C) c = 1;
        else
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                if (strong[e] && cf[ci[e]] == ORC_C) ++c;
        prp[i + 1] = prp[i] + c;
    }
    int32_t nnz = prp[n];
    int32_t *pci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *pv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!pci || !pv) { free(cmap); free(prp); free(pci); free(pv); return ORC_E_NOMEM; }
    for (int32_t i = 0; i < n; ++i) {
        int32_t o = prp[i];
        if (cf[i] == ORC_C) { pci[o] = cmap[i]; pv[o] = 1.0; continue; }
        if (prp[i + 1] == o) continue;
        double d = 0.0, num = 0.0, den = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] == i) d = v[e];
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] == i) continue;
            if (v[e] > 0.0) d = d + v[e];
            else if (v[e] < 0.0) num = num + v[e];
        }
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (strong[e] && cf[ci[e]] == ORC_C) den = den + v[e];
        double alpha = num / den;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (strong[e] && cf[ci[e]] == ORC_C) {
                pci[o] = cmap[ci[e]];
                pv[o] = -(alpha * v[e]) / d;
                ++o;
            }
    }
    free(cmap);
    P->nrows = n; P->ncols = nc; P->rp = prp; P->ci = pci; P->val = pv;
    return ORC_OK;
}

/*
 * The paper's classical-AMG interpolations (Section 2, Interpolation), with
 * the neighbour sets defined there for an F point i:
 *   N_i   = off-diagonal neighbours of i (a_ij stored, j != i),
 *   S_i   = strong neighbours (the strength flags of the level),
 *   F_i^S = S_i n F,  C_i^S = S_i n C,  N_i^w = N_i \ (F_i^S u C_i^S),
 * and the sign-filtered entry abar_kl = a_kl unless a_kl has the sign of
 * a_kk, in which case it is 0.
 *
 * Classical (eq. clasInt, with the correction for PMIS coarsenings): the
 * interpolatory set is C_i^S.  A strong F neighbour k whose filtered row
 * has no entry on C_i^S (sum_{m in C_i^S} abar_km = 0) belongs to F_i^{S*}
 * and is lumped into the diagonal together with N_i^w; every other k
 * distributes a_ik over C_i^S in proportion to abar_kj.  The printed
 * numerator lacks the direct coupling a_ij; it is restored here as in the
 * extended+i formula and the Henson-Yang correction the paper follows, so
 * that rows with zero sum interpolate constants exactly.
 *
 * Extended+i (eq. extpiInt): the set is C^_i = C_i^S u (union over k in
 * F_i^S of C_k^S), k's share is spread over C^_i u {i}, the part that falls
 * on i itself moves into the diagonal a~_ii, and weak neighbours outside
 * C^_i are lumped.  A k whose filtered row has no entry on C^_i u {i} (its
 * share cannot be spread) is lumped into the diagonal as well.
 *
 * Hybrid: the same formula on the smaller set C^h_i of Alg. extintset:
 * start from C_i^S; F' = strong F neighbours with no strong connection to
 * the set (k strongly depends on no point of it) that have at least one
 * strong C neighbour; repeatedly add the candidate C point (a strong C
 * neighbour of some point of F') that covers the most points of F', the
 * smallest index on ties, and drop the points it covers from F'.  The loop
 * ends when F' is empty.
 *
 * C rows are identity rows; an F row with an empty set is an empty row.
 * Sums run in CSR order of row i, the set in ascending order.
 */
static double abar(const int32_t *rp, const int32_t *ci, const double *v, int32_t k, int32_t l) {
    int32_t e = find_in_row(rp, ci, k, l);
    if (e < 0) return 0.0;
    int32_t d = find_in_row(rp, ci, k, k);
    double akk = v[d], a = v[e];
    int sa = (a > 0.0) - (a < 0.0), sd = (akk > 0.0) - (akk < 0.0);
    return sa == sd ? 0.0 : a;
}

/* l in S_k: k strongly depends on l */
static int depends(const int32_t *rp, const int32_t *ci, const uint8_t *strong, int32_t k, int32_t l) {
    int32_t e = find_in_row(rp, ci, k, l);
    return e >= 0 && strong[e];
}

static int is_strong_f(const int32_t *ci, const uint8_t *strong, const int8_t *cf, int32_t i, int32_t e) {
    return ci[e] != i && strong[e] && cf[ci[e]] == ORC_F;
}

/* Interpolatory set of F point i, ascending, in set[0..*ns); mark[c] == i
 * flags its members.  set, fp and mark hold n entries each. */
static void interp_set(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong, const int8_t *cf,
                       int32_t variant, int32_t i, int32_t *set, int32_t *ns, int32_t *fp, int32_t *mark) {
    (void)n;
    int32_t m = 0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] != i && strong[e] && cf[ci[e]] == ORC_C) { set[m++] = ci[e]; mark[ci[e]] = i; }
    if (variant == ORC_INTERP_EXTI) {
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (!is_strong_f(ci, strong, cf, i, e)) continue;
            int32_t k = ci[e];
            for (int32_t f = rp[k]; f < rp[k + 1]; ++f) {
                int32_t c = ci[f];
                if (c != k && strong[f] && cf[c] == ORC_C && mark[c] != i) { set[m++] = c; mark[c] = i; }
            }
        }
    } else if (variant == ORC_INTERP_HYBRID) {
        int32_t nf = 0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (!is_strong_f(ci, strong, cf, i, e)) continue;
            int32_t k = ci[e], covered = 0, has_c = 0;
            for (int32_t f = rp[k]; f < rp[k + 1]; ++f) {
                int32_t c = ci[f];
                if (c == k || !strong[f] || cf[c] != ORC_C) continue;
                has_c = 1;
                if (mark[c] == i) covered = 1;
            }
            if (has_c && !covered) fp[nf++] = k;
        }
        while (nf > 0) {
            int32_t best = -1, bestdeg = 0;
            for (int32_t a = 0; a < nf; ++a) {
                int32_t k = fp[a];
                for (int32_t f = rp[k]; f < rp[k + 1]; ++f) {
                    int32_t c = ci[f];
                    if (c == k || !strong[f] || cf[c] != ORC_C) continue;
                    int32_t deg = 0;
                    for (int32_t b = 0; b < nf; ++b) deg += depends(rp, ci, strong, fp[b], c);
                    if (deg > bestdeg || (deg == bestdeg && c < best)) { best = c; bestdeg = deg; }
                }
            }
            set[m++] = best;
            mark[best] = i;
            int32_t keep = 0;
            for (int32_t a = 0; a < nf; ++a)
                if (!depends(rp, ci, strong, fp[a], best)) fp[keep++] = fp[a];
            nf = keep;
        }
    }
    qsort(set, (size_t)m, sizeof(int32_t), cmp_i32);
    *ns = m;
}

int orc_interp(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const uint8_t *strong,
               const int8_t *cf, int32_t variant, orc_csr *P) {
    if (variant == ORC_INTERP_DIRECT) return orc_interp_direct(n, rp, ci, v, strong, cf, P);
    if (variant != ORC_INTERP_CLASSICAL && variant != ORC_INTERP_EXTI && variant != ORC_INTERP_HYBRID)
        return ORC_E_ARG;
    int32_t *cmap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *set = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *fp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *num = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *prp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *pci = NULL;
    double *pv = NULL;
    if (!cmap || !mark || !set || !fp || !num || !prp) goto nomem;
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i) { cmap[i] = nc; if (cf[i] == ORC_C) ++nc; mark[i] = -1; }
    prp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t ns = 1;
        if (cf[i] != ORC_C) interp_set(n, rp, ci, strong, cf, variant, i, set, &ns, fp, mark);
        prp[i + 1] = prp[i] + ns;
    }
    int32_t nnz = prp[n];
    pci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    pv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!pci || !pv) goto nomem;
    for (int32_t i = 0; i < n; ++i) mark[i] = -1;
    int plus_i = variant != ORC_INTERP_CLASSICAL;
    for (int32_t i = 0; i < n; ++i) {
        int32_t o = prp[i];
        if (cf[i] == ORC_C) { pci[o] = cmap[i]; pv[o] = 1.0; continue; }
        int32_t ns = 0;
        interp_set(n, rp, ci, strong, cf, variant, i, set, &ns, fp, mark);
        if (ns == 0) continue;
        for (int32_t t = 0; t < ns; ++t) {
            int32_t e = find_in_row(rp, ci, i, set[t]);
            num[t] = e >= 0 ? v[e] : 0.0;
        }
        double diag = v[find_in_row(rp, ci, i, i)];
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t k = ci[e];
            if (k == i) continue;
            if (is_strong_f(ci, strong, cf, i, e)) {
                /* share of k, spread over the set (and i itself for extended+i and hybrid) */
                double D = 0.0;
                for (int32_t t = 0; t < ns; ++t) {
                    if (plus_i && i < set[t] && (t == 0 || set[t - 1] < i)) D = D + abar(rp, ci, v, k, i);
                    D = D + abar(rp, ci, v, k, set[t]);
                }
                if (plus_i && set[ns - 1] < i) D = D + abar(rp, ci, v, k, i);
                if (D == 0.0) { diag = diag + v[e]; continue; }
                for (int32_t t = 0; t < ns; ++t) num[t] = num[t] + (v[e] * abar(rp, ci, v, k, set[t])) / D;
                if (plus_i) diag = diag + (v[e] * abar(rp, ci, v, k, i)) / D;
            } else if (mark[k] != i) {
                diag = diag + v[e];  /* weak neighbour outside the set */
            }
        }
        for (int32_t t = 0; t < ns; ++t) {
            pci[o + t] = cmap[set[t]];
            pv[o + t] = -num[t] / diag;
        }
    }
    free(cmap); free(mark); free(set); free(fp); free(num);
    P->nrows = n; P->ncols = nc; P->rp = prp; P->ci = pci; P->val = pv;
    return ORC_OK;
nomem:
    free(cmap); free(mark); free(set); free(fp); free(num); free(prp); free(pci); free(pv);
    return ORC_E_NOMEM;
}

/*
 * BAMG prolongation (Section 2, Interpolation, eq. minBAMG and Alg. BAMG)
 * for a given test space V (n x nt, row k = phi_k).
 *
 * Orthonormal basis of the test space: Cholesky-QR, G = V^T V (each entry
 * summed over rows in index order), G = L L^T, V <- V L^{-T} row by row.
 * A pivot at or below 1e-12 of the largest diagonal entry of G (a column
 * whose independent part is below 1e-6 of the largest column) is an error.
 */
int orc_orthonormalize(int32_t n, int32_t nt, double *V) {
    if (nt < 1 || nt > ORC_MAXNT) return ORC_E_ARG;
    double G[ORC_MAXNT * ORC_MAXNT];
    for (int32_t a = 0; a < nt; ++a)
        for (int32_t b = 0; b <= a; ++b) {
            double s = 0.0;
            for (int32_t r = 0; r < n; ++r) s = s + V[(size_t)r * nt + a] * V[(size_t)r * nt + b];
            G[a * nt + b] = s;
        }
    double gmax = 0.0;
    for (int32_t a = 0; a < nt; ++a) gmax = G[a * nt + a] > gmax ? G[a * nt + a] : gmax;
    /* G = L L^T (lower triangle, column by column) */
    for (int32_t j = 0; j < nt; ++j) {
        double d = G[j * nt + j];
        for (int32_t k = 0; k < j; ++k) d = d - G[j * nt + k] * G[j * nt + k];
        if (!(d > 1e-12 * gmax)) return ORC_E_ARG;  /* independent part below 1e-6 of the largest column */
        double ljj = sqrt(d);
        G[j * nt + j] = ljj;
        for (int32_t i = j + 1; i < nt; ++i) {
            double t = G[i * nt + j];
            for (int32_t k = 0; k < j; ++k) t = t - G[i * nt + k] * G[j * nt + k];
            G[i * nt + j] = t / ljj;
        }
    }
    /* each row x of V becomes the solution y of L y = x */
    for (int32_t r = 0; r < n; ++r) {
        double *x = V + (size_t)r * nt;
        for (int32_t a = 0; a < nt; ++a) {
            double t = x[a];
            for (int32_t k = 0; k < a; ++k) t = t - G[a * nt + k] * x[k];
            x[a] = t / G[a * nt + a];
        }
    }
    return ORC_OK;
}

/*
 * Interpolatory candidates of F point i at distance l: the C points reached
 * from i by at most l steps along strong connections (k -> j for j in S_k),
 * ascending.  mark (n entries, -1 outside a call) flags visited points,
 * dist their distance; front lists them.
 */
static int32_t bamg_candidates(const int32_t *rp, const int32_t *ci, const uint8_t *strong, const int8_t *cf,
                               int32_t i, int32_t l, int32_t *mark, int32_t *dist, int32_t *front, int32_t *cand) {
    int32_t nf = 1, nc = 0, head = 0;
    front[0] = i;
    mark[i] = i;
    dist[i] = 0;
    while (head < nf) {
        int32_t k = front[head++];
        if (dist[k] == l) continue;
        for (int32_t e = rp[k]; e < rp[k + 1]; ++e) {
            int32_t j = ci[e];
            if (j == k || !strong[e] || mark[j] == i) continue;
            mark[j] = i;
            dist[j] = dist[k] + 1;
            front[nf++] = j;
            if (cf[j] == ORC_C) cand[nc++] = j;
        }
    }
    for (int32_t t = 0; t < nf; ++t) mark[front[t]] = -1;
    qsort(cand, (size_t)nc, sizeof(int32_t), cmp_i32);
    return nc;
}

/*
 * Weights of row i over the candidates cand[0..nc) (eq. minBAMG): a basis of
 * the candidates' test-space rows is chosen greedily (maxvol by pivoted
 * modified Gram-Schmidt: at each step the candidate whose residual row has
 * the largest norm, the smallest index on ties, until nt are chosen or the
 * largest residual is below 1e-10 of the largest row norm), phi_i is
 * projected on the orthonormal q's (c_m = q_m . res, res -= c_m q_m), and
 * R w = c is solved (R from the pivoted Gram-Schmidt).  Outputs the chosen
 * candidates sel[0..r) (in choice order), w, the relative residual and
 * ||w||.
 */
static int32_t bamg_weights(int32_t nt, const double *V, int32_t i, const int32_t *cand, int32_t nc, double *work,
                            double *coef, int32_t *sel, double *w, double *relres, double *wnorm) {
    double q[ORC_MAXNT][ORC_MAXNT], R[ORC_MAXNT][ORC_MAXNT], c[ORC_MAXNT], res[ORC_MAXNT];
    uint8_t used[ORC_MAXCAND];
    double n0 = 0.0;
    for (int32_t t = 0; t < nc; ++t) {
        used[t] = 0;
        double s = 0.0;
        for (int32_t a = 0; a < nt; ++a) {
            work[t * nt + a] = V[(size_t)cand[t] * nt + a];
            s = s + work[t * nt + a] * work[t * nt + a];
        }
        n0 = s > n0 ? s : n0;
    }
    int32_t r = 0;
    while (r < nt) {
        int32_t best = -1;
        double bn = 0.0;
        for (int32_t t = 0; t < nc; ++t) {
            if (used[t]) continue;
            double s = 0.0;
            for (int32_t a = 0; a < nt; ++a) s = s + work[t * nt + a] * work[t * nt + a];
            if (s > bn) { bn = s; best = t; }
        }
        if (best < 0 || !(bn > 1e-20 * n0)) break;
        double nb = sqrt(bn);
        for (int32_t a = 0; a < nt; ++a) q[r][a] = work[best * nt + a] / nb;
        for (int32_t m = 0; m < r; ++m) R[m][r] = coef[best * nt + m];
        R[r][r] = nb;
        used[best] = 1;
        sel[r] = best;
        for (int32_t t = 0; t < nc; ++t) {
            if (used[t]) continue;
            double d = 0.0;
            for (int32_t a = 0; a < nt; ++a) d = d + q[r][a] * work[t * nt + a];
            coef[t * nt + r] = d;
            for (int32_t a = 0; a < nt; ++a) work[t * nt + a] = work[t * nt + a] - d * q[r][a];
        }
        ++r;
    }
    double ni = 0.0;
    for (int32_t a = 0; a < nt; ++a) {
        res[a] = V[(size_t)i * nt + a];
        ni = ni + res[a] * res[a];
    }
    for (int32_t m = 0; m < r; ++m) {
        double d = 0.0;
        for (int32_t a = 0; a < nt; ++a) d = d + q[m][a] * res[a];
        c[m] = d;
        for (int32_t a = 0; a < nt; ++a) res[a] = res[a] - d * q[m][a];
    }
    for (int32_t m = r - 1; m >= 0; --m) {
        double t = c[m];
        for (int32_t k = m + 1; k < r; ++k) t = t - R[m][k] * w[k];
        w[m] = t / R[m][m];
    }
    double nr = 0.0, nw = 0.0;
    for (int32_t a = 0; a < nt; ++a) nr = nr + res[a] * res[a];
    for (int32_t m = 0; m < r; ++m) nw = nw + w[m] * w[m];
    *relres = ni > 0.0 ? sqrt(nr) / sqrt(ni) : 0.0;
    *wnorm = sqrt(nw);
    return r;
}

/*
 * Alg. BAMG over the F points (its printed loop over C points is read as
 * over F points; C rows are identity rows): from l = lmin, take the
 * candidates at distance <= l, their weights, and stop when the relative
 * residual is <= eps and ||w|| <= mu, or at l = lmax.  The row lists the
 * chosen candidates in ascending order; no candidate gives an empty row.
 * More than ORC_MAXCAND candidates is an error.
 */
int orc_bamg(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong, const int8_t *cf, int32_t nt,
             const double *V, int32_t lmin, int32_t lmax, double eps, double mu, orc_csr *P) {
    if (nt < 1 || nt > ORC_MAXNT || lmin < 1 || lmax < lmin) return ORC_E_ARG;
    int32_t *cmap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *front = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *work = (double *)malloc(sizeof(double) * (size_t)ORC_MAXCAND * nt);
    double *coef = (double *)malloc(sizeof(double) * (size_t)ORC_MAXCAND * nt);
    int32_t *prp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *pci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n * nt + 1));
    double *pv = (double *)malloc(sizeof(double) * ((size_t)n * nt + 1));
    int st = ORC_OK;
    if (!cmap || !mark || !dist || !front || !cand || !work || !coef || !prp || !pci || !pv) { st = ORC_E_NOMEM; goto done; }
    int32_t nc0 = 0;
    for (int32_t i = 0; i < n; ++i) { cmap[i] = nc0; if (cf[i] == ORC_C) ++nc0; mark[i] = -1; }
    prp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t o = prp[i];
        if (cf[i] == ORC_C) { pci[o] = cmap[i]; pv[o] = 1.0; prp[i + 1] = o + 1; continue; }
        int32_t sel[ORC_MAXNT], r = 0, nc = 0;
        double w[ORC_MAXNT], relres = 0.0, wn = 0.0;
        for (int32_t l = lmin; l <= lmax; ++l) {
            nc = bamg_candidates(rp, ci, strong, cf, i, l, mark, dist, front, cand);
            if (nc > ORC_MAXCAND) { st = ORC_E_ARG; goto done; }
            r = nc > 0 ? bamg_weights(nt, V, i, cand, nc, work, coef, sel, w, &relres, &wn) : 0;
            if (relres <= eps && wn <= mu && r > 0) break;
        }
        /* ascending candidate order */
        int32_t ord[ORC_MAXNT];
        for (int32_t m = 0; m < r; ++m) ord[m] = m;
        for (int32_t a = 1; a < r; ++a) {
            int32_t x = ord[a], b = a - 1;
            while (b >= 0 && cand[sel[ord[b]]] > cand[sel[x]]) { ord[b + 1] = ord[b]; --b; }
            ord[b + 1] = x;
        }
        for (int32_t m = 0; m < r; ++m) {
            pci[o + m] = cmap[cand[sel[ord[m]]]];
            pv[o + m] = w[ord[m]];
        }
        prp[i + 1] = o + r;
    }
    P->nrows = n; P->ncols = nc0; P->rp = prp; P->ci = pci; P->val = pv;
    prp = NULL; pci = NULL; pv = NULL;
done:
    free(cmap); free(mark); free(dist); free(front); free(cand); free(work); free(coef);
    free(prp); free(pci); free(pv);
    return st;
}

/*
 * Prolongation smoothing (Section 2, Interpolation, end): one Jacobi step
 * on the columns of P, Ps = P - omega D^{-1} (A P), with the level's Jacobi
 * weight; row i holds the union of the patterns of P and A P (ascending),
 * entry p - (omega dinv_i) ap with a missing entry read as 0.
 */
int orc_psmooth(const orc_csr *A, const double *dinv, double omega, const orc_csr *P, orc_csr *Ps) {
    orc_csr AP = {0, 0, NULL, NULL, NULL};
    int st = orc_spgemm(A, P, &AP);
    if (st) return st;
    int32_t n = P->nrows;
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t cap = P->rp[n] + AP.rp[n];
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    double *val = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
    if (!rp || !ci || !val) { free(rp); free(ci); free(val); orc_csr_free(&AP); return ORC_E_NOMEM; }
    int32_t o = 0;
    rp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        double s = omega * dinv[i];
        int32_t a = P->rp[i], b = AP.rp[i];
        while (a < P->rp[i + 1] || b < AP.rp[i + 1]) {
            int32_t ja = a < P->rp[i + 1] ? P->ci[a] : INT32_MAX;
            int32_t jb = b < AP.rp[i + 1] ? AP.ci[b] : INT32_MAX;
            int32_t j = ja < jb ? ja : jb;
            double pv = 0.0, av = 0.0;
            if (ja == j) pv = P->val[a++];
            if (jb == j) av = AP.val[b++];
            ci[o] = j;
            val[o] = pv - s * av;
            ++o;
        }
        rp[i + 1] = o;
    }
    orc_csr_free(&AP);
    Ps->nrows = n; Ps->ncols = P->ncols; Ps->rp = rp; Ps->ci = ci; Ps->val = val;
    return ORC_OK;
}

/*
 * Filtering of P with compensation (Section 2, Filtering, eq. action): per
 * row, the entries are ranked by decreasing |p| (the smaller column first on
 * ties) and the shortest leading set whose absolute sum (added in that
 * order) reaches rho times the row's absolute sum is kept.  The dropped
 * entries' action on the coarse test space W (nc x nt), r = sum over the
 * dropped entries (ascending column) of p_j W_j, is moved onto the kept
 * entries K by the minimum-norm correction d = B^T (B B^T + lambda I)^{-1} r,
 * B = [W_k]_{k in K} (nt x |K|, kept entries in ascending column), lambda =
 * 1e-12 trace(B B^T) / nt; the kept entries become p_k + d_k.  Then
 * P~ W = P W up to the ridge term.  rho >= 1 keeps every row as it is.
 */
int orc_pfilter(const orc_csr *P, double rho, int32_t nt, const double *W, orc_csr *Pf) {
    int32_t n = P->nrows, nnz = P->rp[n];
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    uint8_t *keep = (uint8_t *)malloc((size_t)(nnz > 0 ? nnz : 1));
    if (!rp || !ci || !val || !ord || !keep) {
        free(rp); free(ci); free(val); free(ord); free(keep);
        return ORC_E_NOMEM;
    }
    int32_t o = 0;
    rp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t e0 = P->rp[i], m = P->rp[i + 1] - e0;
        const int32_t *pc = P->ci + e0;
        const double *pv = P->val + e0;
        for (int32_t t = 0; t < m; ++t) keep[t] = 1;
        if (rho < 1.0 && m > 1) {
            /* rank by |p| descending, column ascending on ties (insertion sort) */
            for (int32_t t = 0; t < m; ++t) {
                int32_t x = t, u = t - 1;
                while (u >= 0 && (fabs(pv[ord[u]]) < fabs(pv[x]) ||
                                  (fabs(pv[ord[u]]) == fabs(pv[x]) && pc[ord[u]] > pc[x]))) {
                    ord[u + 1] = ord[u];
                    --u;
                }
                ord[u + 1] = x;
            }
            double tot = 0.0, run = 0.0;
            for (int32_t t = 0; t < m; ++t) tot = tot + fabs(pv[ord[t]]);
            int32_t nk = 0;
            while (nk < m && run < rho * tot) run = run + fabs(pv[ord[nk++]]);
            if (nk < 1) nk = 1;
            for (int32_t t = 0; t < m; ++t) keep[t] = 0;
            for (int32_t t = 0; t < nk; ++t) keep[ord[t]] = 1;
        }
        /* action of the dropped entries on W */
        double r[ORC_MAXNT], G[ORC_MAXNT * ORC_MAXNT], y[ORC_MAXNT];
        int32_t dropped = 0;
        for (int32_t a = 0; a < nt; ++a) r[a] = 0.0;
        for (int32_t t = 0; t < m; ++t)
            if (!keep[t]) {
                dropped = 1;
                for (int32_t a = 0; a < nt; ++a) r[a] = r[a] + pv[t] * W[(size_t)pc[t] * nt + a];
            }
        if (dropped) {
            for (int32_t a = 0; a < nt; ++a)
                for (int32_t b = 0; b <= a; ++b) {
                    double g = 0.0;
                    for (int32_t t = 0; t < m; ++t)
                        if (keep[t]) g = g + W[(size_t)pc[t] * nt + a] * W[(size_t)pc[t] * nt + b];
                    G[a * nt + b] = g;
                }
            double tr = 0.0;
            for (int32_t a = 0; a < nt; ++a) tr = tr + G[a * nt + a];
            double lam = 1e-12 * tr / nt;
            for (int32_t a = 0; a < nt; ++a) G[a * nt + a] = G[a * nt + a] + lam;
            /* (B B^T + lambda I) y = r by Cholesky */
            for (int32_t j = 0; j < nt; ++j) {
                double d = G[j * nt + j];
                for (int32_t k = 0; k < j; ++k) d = d - G[j * nt + k] * G[j * nt + k];
                double ljj = sqrt(d > 0.0 ? d : 0.0);
                G[j * nt + j] = ljj;
                for (int32_t q = j + 1; q < nt; ++q) {
                    double t = G[q * nt + j];
                    for (int32_t k = 0; k < j; ++k) t = t - G[q * nt + k] * G[j * nt + k];
                    G[q * nt + j] = ljj > 0.0 ? t / ljj : 0.0;
                }
            }
            for (int32_t a = 0; a < nt; ++a) {
                double t = r[a];
                for (int32_t k = 0; k < a; ++k) t = t - G[a * nt + k] * y[k];
                y[a] = G[a * nt + a] > 0.0 ? t / G[a * nt + a] : 0.0;
            }
            for (int32_t a = nt - 1; a >= 0; --a) {
                double t = y[a];
                for (int32_t k = a + 1; k < nt; ++k) t = t - G[k * nt + a] * y[k];
                y[a] = G[a * nt + a] > 0.0 ? t / G[a * nt + a] : 0.0;
            }
        }
        for (int32_t t = 0; t < m; ++t) {
            if (!keep[t]) continue;
            double d = 0.0;
            if (dropped)
                for (int32_t a = 0; a < nt; ++a) d = d + W[(size_t)pc[t] * nt + a] * y[a];
            ci[o] = pc[t];
            val[o] = pv[t] + d;
            ++o;
        }
        rp[i + 1] = o;
    }
    free(ord); free(keep);
    Pf->nrows = n; Pf->ncols = P->ncols; Pf->rp = rp; Pf->ci = ci; Pf->val = val;
    return ORC_OK;
}

/*
 * Eigen-decomposition C = Q diag(lam) Q^T of a symmetric m x m matrix
 * (row-major, overwritten) by the cyclic Jacobi method (Golub and Van Loan,
 * Matrix Computations, the classical symmetric Schur rotation): pairs
 * (p, q), p < q, are visited row by row; each rotation zeroes C[p][q] with
 * tau = (c_qq - c_pp) / (2 c_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
 * c = 1 / sqrt(1 + t^2), s = t c, and updates the columns p, q of C, then
 * its rows p, q, then the columns p, q of Q (Q starts as I).  Sweeps stop
 * when the sum of squares above the diagonal is at most 1e-30 times the
 * squared Frobenius norm of the input, or after 60 sweeps.  lam[i] = C[i][i]
 * and column i of Q is its eigenvector.
 */
int orc_symeig(int32_t m, double *C, double *lam, double *Q) {
    if (m < 1 || m > 2 * ORC_MAXNT) return ORC_E_ARG;
    double tot = 0.0;
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < m; ++j) tot = tot + C[i * m + j] * C[i * m + j];
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < m; ++j) Q[i * m + j] = i == j ? 1.0 : 0.0;
    for (int32_t sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int32_t p = 0; p < m; ++p)
            for (int32_t q = p + 1; q < m; ++q) off = off + C[p * m + q] * C[p * m + q];
        if (!(off > 1e-30 * tot)) break;
        for (int32_t p = 0; p < m; ++p)
            for (int32_t q = p + 1; q < m; ++q) {
                const double apq = C[p * m + q];
                if (apq == 0.0) continue;
                const double tau = (C[q * m + q] - C[p * m + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                for (int32_t k = 0; k < m; ++k) {
                    const double x = C[k * m + p], y = C[k * m + q];
                    C[k * m + p] = c * x - s * y;
                    C[k * m + q] = s * x + c * y;
                }
                for (int32_t k = 0; k < m; ++k) {
                    const double x = C[p * m + k], y = C[q * m + k];
                    C[p * m + k] = c * x - s * y;
                    C[q * m + k] = s * x + c * y;
                }
                for (int32_t k = 0; k < m; ++k) {
                    const double x = Q[k * m + p], y = Q[k * m + q];
                    Q[k * m + p] = c * x - s * y;
                    Q[k * m + q] = s * x + c * y;
                }
            }
    }
    for (int32_t i = 0; i < m; ++i) lam[i] = C[i * m + i];
    return ORC_OK;
}

/* Y = A X for a block of k columns: row i of Y (stride ldy) is the sum, over
 * the entries of row i of A in order, of a_ij times row j of X (stride ldx). */
static void csr_block(const orc_csr *A, int32_t k, const double *X, int32_t ldx, double *Y, int32_t ldy) {
    for (int32_t i = 0; i < A->nrows; ++i) {
        for (int32_t a = 0; a < k; ++a) Y[(size_t)i * ldy + a] = 0.0;
        for (int32_t e = A->rp[i]; e < A->rp[i + 1]; ++e) {
            const double aij = A->val[e];
            const double *x = X + (size_t)A->ci[e] * ldx;
            for (int32_t a = 0; a < k; ++a) Y[(size_t)i * ldy + a] = Y[(size_t)i * ldy + a] + aij * x[a];
        }
    }
}

/*
 * Test-space refinement by simultaneous Rayleigh quotient minimisation
 * (Section 2, Unveiling the operator near kernel, eq. eigP), preconditioned
 * with the level's smoother: M^{-1} = D^{-1} (Jacobi; G = NULL) or
 * M^{-1} = G^T G (FSAI).  The paper fixes the method and the preconditioner,
 * not the update; read as block preconditioned steepest descent with
 * Rayleigh-Ritz (the trace of V^T A V is minimised over span[V, W]):
 *
 *   X = A V, T = V^T X, R = X - V T, W = M^{-1} R, S = [V W] (n x 2nt),
 *   Gs = S^T S, Hs = S^T (A S)  (lower triangles, sums over rows in order),
 *   Cholesky of Gs row by row, leaving out a column of S whose pivot is at
 *   most 1e-12 times the largest diagonal of Gs (it adds no direction),
 *   C = L^{-1} Hs L^{-T} on the kept columns, C = Q diag(lam) Q^T,
 *   the nt smallest lam (the smaller index on ties), Z = L^{-T} Q_sel,
 *   V = S_kept Z.
 *
 * V (n x nt, row-major, orthonormal on input) is updated in place for at
 * most iters steps; a step in which every column of W is left out ends the
 * iteration with V unchanged.  *done receives the number of steps taken.
 */
int orc_srqm(const orc_csr *A, const double *dinv, const orc_csr *G, const orc_csr *GT, int32_t nt, double *V,
             int32_t iters, int32_t *done) {
    *done = 0;
    if (nt < 1 || nt > ORC_MAXNT || iters < 0) return ORC_E_ARG;
    const int32_t n = A->nrows, m = 2 * nt;
    double *S = (double *)malloc(sizeof(double) * ((size_t)n * m + 1));
    double *AS = (double *)malloc(sizeof(double) * ((size_t)n * m + 1));
    double *R = (double *)malloc(sizeof(double) * ((size_t)n * nt + 1));
    double *Y = (double *)malloc(sizeof(double) * ((size_t)n * nt + 1));
    if (!S || !AS || !R || !Y) { free(S); free(AS); free(R); free(Y); return ORC_E_NOMEM; }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = 0; a < nt; ++a) S[(size_t)i * m + a] = V[(size_t)i * nt + a];
    double T[ORC_MAXNT * ORC_MAXNT];
    double Gs[4 * ORC_MAXNT * ORC_MAXNT], Hs[4 * ORC_MAXNT * ORC_MAXNT], L[4 * ORC_MAXNT * ORC_MAXNT];
    double Cm[4 * ORC_MAXNT * ORC_MAXNT], Q[4 * ORC_MAXNT * ORC_MAXNT], lam[2 * ORC_MAXNT];
    double Z[2 * ORC_MAXNT * ORC_MAXNT];
    int32_t K[2 * ORC_MAXNT];
    for (int32_t it = 0; it < iters; ++it) {
        /* X = A V into the first nt columns of AS */
        csr_block(A, nt, S, m, AS, m);
        /* T = V^T X, R = X - V T */
        for (int32_t a = 0; a < nt; ++a)
            for (int32_t b = 0; b < nt; ++b) {
                double s = 0.0;
                for (int32_t i = 0; i < n; ++i) s = s + S[(size_t)i * m + a] * AS[(size_t)i * m + b];
                T[a * nt + b] = s;
            }
        for (int32_t i = 0; i < n; ++i)
            for (int32_t b = 0; b < nt; ++b) {
                double r = AS[(size_t)i * m + b];
                for (int32_t a = 0; a < nt; ++a) r = r - S[(size_t)i * m + a] * T[a * nt + b];
                R[(size_t)i * nt + b] = r;
            }
        /* W = M^{-1} R into the last nt columns of S */
        if (G) {
            csr_block(G, nt, R, nt, Y, nt);
            csr_block(GT, nt, Y, nt, S + nt, m);
        } else {
            for (int32_t i = 0; i < n; ++i)
                for (int32_t b = 0; b < nt; ++b) S[(size_t)i * m + nt + b] = dinv[i] * R[(size_t)i * nt + b];
        }
        csr_block(A, nt, S + nt, m, AS + nt, m);
        /* Gram matrices of the subspace (lower triangles, mirrored) */
        for (int32_t a = 0; a < m; ++a)
            for (int32_t b = 0; b <= a; ++b) {
                double g = 0.0, h = 0.0;
                for (int32_t i = 0; i < n; ++i) g = g + S[(size_t)i * m + a] * S[(size_t)i * m + b];
                for (int32_t i = 0; i < n; ++i) h = h + S[(size_t)i * m + a] * AS[(size_t)i * m + b];
                Gs[a * m + b] = g; Gs[b * m + a] = g;
                Hs[a * m + b] = h; Hs[b * m + a] = h;
            }
        /* Cholesky of Gs, row by row, leaving out dependent columns */
        double gmax = 0.0;
        for (int32_t a = 0; a < m; ++a) gmax = Gs[a * m + a] > gmax ? Gs[a * m + a] : gmax;
        int32_t mk = 0;
        for (int32_t j = 0; j < m; ++j) {
            for (int32_t k = 0; k < mk; ++k) {
                double t = Gs[j * m + K[k]];
                for (int32_t q = 0; q < k; ++q) t = t - L[mk * m + q] * L[k * m + q];
                L[mk * m + k] = t / L[k * m + k];
            }
            double d = Gs[j * m + j];
            for (int32_t k = 0; k < mk; ++k) d = d - L[mk * m + k] * L[mk * m + k];
            if (!(d > 1e-12 * gmax)) continue;
            L[mk * m + mk] = sqrt(d);
            K[mk] = j;
            ++mk;
        }
        if (mk <= nt) break;  /* W adds nothing to span V */
        /* C = L^{-1} Hs L^{-T}: first Cm = L^{-1} Hs (columns by forward
         * substitution), then C = L^{-1} Cm^T, lower triangle mirrored */
        for (int32_t c = 0; c < mk; ++c)
            for (int32_t r = 0; r < mk; ++r) {
                double t = Hs[K[r] * m + K[c]];
                for (int32_t q = 0; q < r; ++q) t = t - L[r * m + q] * Cm[q * m + c];
                Cm[r * m + c] = t / L[r * m + r];
            }
        for (int32_t c = 0; c < mk; ++c)
            for (int32_t r = 0; r < mk; ++r) {
                double t = Cm[c * m + r];
                for (int32_t q = 0; q < r; ++q) t = t - L[r * m + q] * Q[q * mk + c];
                Q[r * mk + c] = t / L[r * m + r];
            }
        for (int32_t r = 0; r < mk; ++r)
            for (int32_t c = 0; c <= r; ++c) {
                Cm[r * mk + c] = Q[r * mk + c];
                Cm[c * mk + r] = Q[r * mk + c];
            }
        orc_symeig(mk, Cm, lam, Q);
        /* the nt smallest Ritz values; Z = L^{-T} Q_sel by back substitution */
        int32_t used[2 * ORC_MAXNT];
        for (int32_t k = 0; k < mk; ++k) used[k] = 0;
        for (int32_t b = 0; b < nt; ++b) {
            int32_t best = -1;
            for (int32_t k = 0; k < mk; ++k)
                if (!used[k] && (best < 0 || lam[k] < lam[best])) best = k;
            used[best] = 1;
            for (int32_t r = mk - 1; r >= 0; --r) {
                double t = Q[r * mk + best];
                for (int32_t q = r + 1; q < mk; ++q) t = t - L[q * m + r] * Z[q * nt + b];
                Z[r * nt + b] = t / L[r * m + r];
            }
        }
        /* V = S_kept Z */
        for (int32_t i = 0; i < n; ++i) {
            double row[2 * ORC_MAXNT];
            for (int32_t k = 0; k < mk; ++k) row[k] = S[(size_t)i * m + K[k]];
            for (int32_t b = 0; b < nt; ++b) {
                double t = 0.0;
                for (int32_t k = 0; k < mk; ++k) t = t + row[k] * Z[k * nt + b];
                S[(size_t)i * m + b] = t;
            }
        }
        *done = it + 1;
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = 0; a < nt; ++a) V[(size_t)i * nt + a] = S[(size_t)i * m + a];
    free(S); free(AS); free(R); free(Y);
    return ORC_OK;
}

/* X^T by counting sort on the column index; rows of the result list their
 * columns in ascending order.  The restriction is R = P^T (eq. AcDef). */
int orc_transpose(const orc_csr *X, orc_csr *XT) {
    int32_t m = X->nrows, nc = X->ncols, nnz = X->rp[m];
    int32_t *rp = (int32_t *)calloc((size_t)nc + 1, sizeof(int32_t));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    if (!rp || !ci || !val || !fill) { free(rp); free(ci); free(val); free(fill); return ORC_E_NOMEM; }
    for (int32_t e = 0; e < nnz; ++e) rp[X->ci[e] + 1] += 1;
    for (int32_t c = 0; c < nc; ++c) rp[c + 1] += rp[c];
    for (int32_t c = 0; c <= nc; ++c) fill[c] = rp[c];
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = X->rp[i]; e < X->rp[i + 1]; ++e) {
            int32_t c = X->ci[e];
            ci[fill[c]] = i;
            val[fill[c]] = X->val[e];
            fill[c] += 1;
        }
    free(fill);
    XT->nrows = nc; XT->ncols = m; XT->rp = rp; XT->ci = ci; XT->val = val;
    return ORC_OK;
}


/*
 * Z = X Y, row by row with a dense accumulator (Gustavson).  The pattern is
 * the full symbolic product: every column reached by a product is kept,
 * even when the values cancel.  For each output entry the products are
 * added in ascending order of the inner index k, starting from 0.0.
 * Used twice to form the Galerkin operator A_c = P^T (A P) (eq. AcDef).
 */
int orc_spgemm(const orc_csr *X, const orc_csr *Y, orc_csr *Z) {
    int32_t m = X->nrows, nc = Y->ncols;
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
    if (!mark || !acc || !cols || !rp) { free(mark); free(acc); free(cols); free(rp); return ORC_E_NOMEM; }
    for (int32_t j = 0; j < nc; ++j) mark[j] = -1;
    /* symbolic */
    int64_t total = 0;
    rp[0] = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t cnt = 0;
        for (int32_t e = X->rp[i]; e < X->rp[i + 1]; ++e) {
            int32_t k = X->ci[e];
            for (int32_t t = Y->rp[k]; t < Y->rp[k + 1]; ++t) {
                int32_t j = Y->ci[t];
                if (mark[j] != i) { mark[j] = i; ++cnt; }
            }
        }
        total += cnt;
        if (total > 2147483647LL) { free(mark); free(acc); free(cols); free(rp); return ORC_E_NOMEM; }
        rp[i + 1] = (int32_t)total;
    }
    int32_t nnz = rp[m];
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!ci || !val) { free(mark); free(acc); free(cols); free(rp); free(ci); free(val); return ORC_E_NOMEM; }
    for (int32_t j = 0; j < nc; ++j) mark[j] = -1;
    /* numeric */
    for (int32_t i = 0; i < m; ++i) {
        int32_t cnt = 0;
        for (int32_t e = X->rp[i]; e < X->rp[i + 1]; ++e) {
            int32_t k = X->ci[e];
            double x = X->val[e];
            for (int32_t t = Y->rp[k]; t < Y->rp[k + 1]; ++t) {
                int32_t j = Y->ci[t];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[cnt++] = j; }
                acc[j] = acc[j] + x * Y->val[t];
            }
        }
        qsort(cols, (size_t)cnt, sizeof(int32_t), cmp_i32);
        for (int32_t q = 0; q < cnt; ++q) {
            ci[rp[i] + q] = cols[q];
            val[rp[i] + q] = acc[cols[q]];
        }
    }
    free(mark); free(acc); free(cols);
    Z->nrows = m; Z->ncols = nc; Z->rp = rp; Z->ci = ci; Z->val = val;
    return ORC_OK;
}

/*
 * Dense Cholesky A = L L^T for the last level (Alg. AMG Set-up: a direct
 * factorisation once the level is small).  Column-oriented: for each column
 * j, the pivot a_jj - sum_k L_jk^2, then the entries below it.  Row-major
 * storage; L overwrites the lower triangle and the strict upper triangle is
 * zeroed.  Returns -(j+1) if pivot j is not positive.
 */
int orc_cholesky(int32_t n, double *a) {
    for (int32_t j = 0; j < n; ++j) {
        double s = a[(size_t)j * n + j];
        for (int32_t k = 0; k < j; ++k) s = s - a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(s > 0.0)) return -(j + 1);
        double ljj = sqrt(s);
        a[(size_t)j * n + j] = ljj;
        for (int32_t i = j + 1; i < n; ++i) {
            double t = a[(size_t)i * n + j];
            for (int32_t k = 0; k < j; ++k) t = t - a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = t / ljj;
        }
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) a[(size_t)i * n + j] = 0.0;
    return 0;
}

/* z = (L L^T)^{-1} y by forward then backward substitution (Alg. AMG
 * application in a V-cycle, last level). */
void orc_chol_solve(int32_t n, const double *L, const double *y, double *z) {
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        double t = y[i];
        for (int32_t k = 0; k < i; ++k) t = t - L[(size_t)i * n + k] * w[k];
        w[i] = t / L[(size_t)i * n + i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double t = w[i];
        for (int32_t k = i + 1; k < n; ++k) t = t - L[(size_t)k * n + i] * z[k];
        z[i] = t / L[(size_t)i * n + i];
    }
    free(w);
}

/*
 * Relaxation weight of the Jacobi smoother S = I - omega D^{-1} A
 * (Section 2, eq. smoother), which needs omega rho(D^{-1} A) < 2.  The paper
 * gives no value; the reading taken is omega = (4/3) / rho_hat with the
 * Gershgorin bound rho_hat = max_i (sum_j |a_ij|) / a_ii >= rho(D^{-1} A),
 * so omega rho <= 4/3.  Row sums in CSR order from 0.0.
 */
double orc_gershgorin_omega(int32_t n, const int32_t *rp, const int32_t *ci, const double *v) {
    double rho = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0, d = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            s = s + fabs(v[e]);
            if (ci[e] == i) d = v[e];
        }
        double q = s / d;
        if (q > rho) rho = q;
    }
    return (4.0 / 3.0) / rho;
}


/*
 * Factorised sparse approximate inverse smoother, M^{-1} = G^T G with G
 * lower triangular (Section 2, eq. smo).  The paper builds G adaptively
 * (aFSAI, from another paper); here G is the static factor of Kolotilina
 * and Yeremin on the pattern of the lower triangle of A: for row i, with
 * P_i = {j <= i : a_ij stored} in ascending order (i last), solve
 * A(P_i, P_i) g = e_last by a dense Cholesky factorisation, forward and
 * backward substitution (the dense routines of the last level), and set
 * G(i, P_i) = g / sqrt(g_last), so that G A G^T has a unit diagonal.
 */
/* the largest number of entries on or below the diagonal in a row of A */
static int32_t lower_row_max(const orc_csr *A) {
    int32_t mmax = 0;
    for (int32_t i = 0; i < A->nrows; ++i) {
        int32_t m = 0;
        for (int32_t e = A->rp[i]; e < A->rp[i + 1]; ++e) if (A->ci[e] <= i) ++m;
        if (m > mmax) mmax = m;
    }
    return mmax;
}

int orc_fsai(const orc_csr *A, orc_csr *G) {
    int32_t n = A->nrows;
    G->nrows = n; G->ncols = n;
    G->rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!G->rp) return ORC_E_NOMEM;
    G->rp[0] = 0;
    int32_t mmax = 1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t m = 0;
        for (int32_t e = A->rp[i]; e < A->rp[i + 1]; ++e) if (A->ci[e] <= i) ++m;
        G->rp[i + 1] = G->rp[i] + m;
        if (m > mmax) mmax = m;
    }
    int32_t nnz = G->rp[n];
    G->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    G->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *M = (double *)malloc(sizeof(double) * (size_t)mmax * (size_t)mmax);
    double *e = (double *)malloc(sizeof(double) * (size_t)mmax);
    double *g = (double *)malloc(sizeof(double) * (size_t)mmax);
    int st = ORC_OK;
    if (!G->ci || !G->val || !M || !e || !g) st = ORC_E_NOMEM;
    for (int32_t i = 0; i < n && st == ORC_OK; ++i) {
        int32_t m = G->rp[i + 1] - G->rp[i];
        const int32_t *idx = A->ci + A->rp[i];   /* the first m columns of row i are <= i */
        for (int32_t r = 0; r < m; ++r)
            for (int32_t c = 0; c < m; ++c) {
                int32_t p = find_in_row(A->rp, A->ci, idx[r], idx[c]);
                M[(size_t)r * m + c] = p >= 0 ? A->val[p] : 0.0;
            }
        if (m == 0 || idx[m - 1] != i || orc_cholesky(m, M) != 0) { st = ORC_E_NOT_SPD; break; }
        /* L L^T g = e_last by the last level's forward and backward
         * substitutions */
        for (int32_t r = 0; r < m; ++r) e[r] = r == m - 1 ? 1.0 : 0.0;
        orc_chol_solve(m, M, e, g);
        if (!(g[m - 1] > 0.0)) { st = ORC_E_NOT_SPD; break; }
        double sd = sqrt(g[m - 1]);
        for (int32_t r = 0; r < m; ++r) {
            G->ci[G->rp[i] + r] = idx[r];
            G->val[G->rp[i] + r] = g[r] / sd;
        }
    }
    free(M); free(e); free(g);
    return st;
}

/*
 * Adaptive FSAI factor, the paper's default smoother (Section 2, eq. smo;
 * the adaptive pattern search is that of the FSAI package the paper cites,
 * JanFerSarGam15, in the reading below).  Row i of G minimises the Kaporin
 * functional psi_i(g) = g^T A g over vectors with g_i = 1 supported on a
 * pattern P_i of columns j <= i, and is then scaled by 1/sqrt(psi_i), so
 * that G A G^T has a unit diagonal.  The pattern grows greedily from
 * P_i = {i}; each pass:
 *   1. solve A(P_i, P_i) y = e_last (P_i ascending, i last) by the dense
 *      Cholesky factorisation and substitutions of the last level; the
 *      minimiser is y / y_last and psi_i = 1 / y_last;
 *   2. stop when `steps` growth steps have been taken, or, after a growth
 *      step, when psi_i fell by no more than eps times its previous value;
 *   3. the candidates are the columns j < i outside P_i stored in the rows
 *      of A indexed by P_i; the gradient of psi_i with respect to g_j is
 *      2 (A g)_j, which is proportional (factor 2 / y_last > 0) to
 *      z_j = sum over the entries a_jc of row j with c in P_i of a_jc y_c,
 *      summed in CSR order from 0.0;
 *   4. add to P_i the `step` candidates with the largest |z_j| > 0 (the
 *      smaller j first on ties); when no candidate has z_j != 0, stop.
 * G(i, P_i) = y / sqrt(y_last), the same scaling as the static factor.
 * steps = 0 gives G = D^{-1/2}.  *maxcand receives the largest candidate
 * set of any row and pass (the hierarchy uses Jacobi on a level where it
 * exceeds ORC_AFSAI_MAXCAND).
 */
typedef struct {
    int32_t *pos;     /* place of a column in the pattern, or -1 */
    int32_t *seen;    /* candidate stamp */
    int32_t *cand;
    double *z;
    uint8_t *taken;
    double *M, *e, *y;
    int32_t stamp;
} afsai_work;

static void afsai_work_free(afsai_work *w) {
    free(w->pos); free(w->seen); free(w->cand); free(w->z); free(w->taken); free(w->M); free(w->e); free(w->y);
}

static int afsai_work_init(afsai_work *w, int32_t n, int32_t mcap) {
    size_t nn = (size_t)(n > 0 ? n : 1);
    w->pos = (int32_t *)malloc(sizeof(int32_t) * nn);
    w->seen = (int32_t *)malloc(sizeof(int32_t) * nn);
    w->cand = (int32_t *)malloc(sizeof(int32_t) * nn);
    w->z = (double *)malloc(sizeof(double) * nn);
    w->taken = (uint8_t *)malloc(nn);
    w->M = (double *)malloc(sizeof(double) * (size_t)mcap * (size_t)mcap);
    w->e = (double *)malloc(sizeof(double) * (size_t)mcap);
    w->y = (double *)malloc(sizeof(double) * (size_t)mcap);
    w->stamp = 0;
    if (!w->pos || !w->seen || !w->cand || !w->z || !w->taken || !w->M || !w->e || !w->y) {
        afsai_work_free(w);
        return ORC_E_NOMEM;
    }
    for (int32_t j = 0; j < n; ++j) { w->pos[j] = -1; w->seen[j] = -1; }
    return ORC_OK;
}

/* one row: its pattern P (ascending, i last) and values into P / val, the
 * count into *mout; the largest candidate set into *maxcand */
static int afsai_row(const orc_csr *A, int32_t i, int32_t steps, int32_t step, double eps, afsai_work *w,
                     int32_t *P, double *val, int32_t *mout, int32_t *maxcand) {
    double *M = w->M, *e = w->e, *y = w->y, *z = w->z;
    int32_t *pos = w->pos, *seen = w->seen, *cand = w->cand;
    uint8_t *taken = w->taken;
    int32_t m = 1;
    P[0] = i;
    double psi_prev = 0.0;
    for (int32_t k = 0;; ++k) {
        /* 1. local system on the current pattern */
        for (int32_t r = 0; r < m; ++r)
            for (int32_t c = 0; c < m; ++c) {
                int32_t p = find_in_row(A->rp, A->ci, P[r], P[c]);
                M[(size_t)r * m + c] = p >= 0 ? A->val[p] : 0.0;
            }
        if (orc_cholesky(m, M) != 0) return ORC_E_NOT_SPD;
        for (int32_t r = 0; r + 1 < m; ++r) e[r] = 0.0;
        e[m - 1] = 1.0;
        orc_chol_solve(m, M, e, y);
        if (!(y[m - 1] > 0.0)) return ORC_E_NOT_SPD;
        const double psi = 1.0 / y[m - 1];
        /* 2. stopping tests */
        if (k == steps) break;
        if (k > 0 && psi_prev - psi <= eps * psi_prev) break;
        psi_prev = psi;
        /* 3. candidates and gradient components */
        for (int32_t r = 0; r < m; ++r) pos[P[r]] = r;
        ++w->stamp;
        int32_t nc = 0;
        for (int32_t r = 0; r < m; ++r)
            for (int32_t q = A->rp[P[r]]; q < A->rp[P[r] + 1]; ++q) {
                int32_t j = A->ci[q];
                if (j < i && pos[j] < 0 && seen[j] != w->stamp) { seen[j] = w->stamp; cand[nc++] = j; }
            }
        if (nc > *maxcand) *maxcand = nc;
        for (int32_t t = 0; t < nc; ++t) {
            int32_t j = cand[t];
            double s = 0.0;
            for (int32_t q = A->rp[j]; q < A->rp[j + 1]; ++q) {
                int32_t c = A->ci[q];
                if (pos[c] >= 0) s = s + A->val[q] * y[pos[c]];
            }
            z[t] = s;
            taken[t] = 0;
        }
        for (int32_t r = 0; r < m; ++r) pos[P[r]] = -1;
        /* 4. the `step` largest |z_j| join the pattern */
        int32_t added = 0;
        for (int32_t a = 0; a < step; ++a) {
            int32_t best = -1;
            for (int32_t t = 0; t < nc; ++t) {
                if (taken[t] || z[t] == 0.0) continue;
                if (best < 0 || fabs(z[t]) > fabs(z[best]) ||
                    (fabs(z[t]) == fabs(z[best]) && cand[t] < cand[best])) best = t;
            }
            if (best < 0) break;
            taken[best] = 1;
            /* insert into the ascending pattern (i stays last) */
            int32_t j = cand[best], r = m;
            while (r > 0 && P[r - 1] > j) { P[r] = P[r - 1]; --r; }
            P[r] = j;
            ++m;
            ++added;
        }
        if (added == 0) break;
    }
    const double sd = sqrt(y[m - 1]);
    for (int32_t r = 0; r < m; ++r) val[r] = y[r] / sd;
    *mout = m;
    return ORC_OK;
}

static int afsai_args_ok(int32_t steps, int32_t step, double eps) {
    return !(steps < 0 || step < 1 || (int64_t)steps * step + 1 > ORC_AFSAI_MAXM || !(eps >= 0.0));
}

int orc_afsai(const orc_csr *A, int32_t steps, int32_t step, double eps, orc_csr *G, int32_t *maxcand) {
    int32_t n = A->nrows;
    G->nrows = n; G->ncols = n;
    G->rp = NULL; G->ci = NULL; G->val = NULL;
    *maxcand = 0;
    if (!afsai_args_ok(steps, step, eps)) return ORC_E_ARG;
    const int32_t mcap = steps * step + 1;
    afsai_work w;
    int st = afsai_work_init(&w, n, mcap);
    if (st) return st;
    G->rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *pci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)mcap);
    double *pv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)mcap);
    if (!G->rp || !pci || !pv) st = ORC_E_NOMEM;
    if (!st) G->rp[0] = 0;
    for (int32_t i = 0; i < n && !st; ++i) {
        int32_t m = 0;
        st = afsai_row(A, i, steps, step, eps, &w, pci + (size_t)i * mcap, pv + (size_t)i * mcap, &m, maxcand);
        if (!st) G->rp[i + 1] = G->rp[i] + m;
    }
    if (!st) {
        int32_t nnz = G->rp[n];
        G->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        G->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        if (!G->ci || !G->val) st = ORC_E_NOMEM;
        for (int32_t i = 0; i < n && !st; ++i)
            for (int32_t r = 0; r < G->rp[i + 1] - G->rp[i]; ++r) {
                G->ci[G->rp[i] + r] = pci[(size_t)i * mcap + r];
                G->val[G->rp[i] + r] = pv[(size_t)i * mcap + r];
            }
    }
    free(pci); free(pv);
    afsai_work_free(&w);
    return st;
}

/* the rows sel[0..nsel) only (for sampled checks of large matrices):
 * row t's pattern and values in cols / vals[t * (steps * step + 1) ...],
 * its entry count in cnt[t] */
int orc_afsai_rows(const orc_csr *A, int32_t steps, int32_t step, double eps, int32_t nsel, const int32_t *sel,
                   int32_t *cols, double *vals, int32_t *cnt, int32_t *maxcand) {
    *maxcand = 0;
    if (!afsai_args_ok(steps, step, eps) || nsel < 0) return ORC_E_ARG;
    const int32_t mcap = steps * step + 1;
    for (int32_t t = 0; t < nsel; ++t)
        if (sel[t] < 0 || sel[t] >= A->nrows) return ORC_E_ARG;
    afsai_work w;
    int st = afsai_work_init(&w, A->nrows, mcap);
    if (st) return st;
    for (int32_t t = 0; t < nsel && !st; ++t)
        st = afsai_row(A, sel[t], steps, step, eps, &w, cols + (size_t)t * mcap, vals + (size_t)t * mcap, &cnt[t],
                       maxcand);
    afsai_work_free(&w);
    return st;
}

static void spmv(const orc_csr *A, const double *s, double *t);

/*
 * Relaxation weight of the FSAI smoother S = I - omega G^T G A, which needs
 * omega rho(G^T G A) < 2 (eq. smoother).  rho(G^T G A) = rho(M) for the
 * symmetric positive definite M = G A G^T.  The paper gives no value; the
 * reading taken is omega = (4/3) / rho_hat, rho_hat the Rayleigh quotient
 * v^T M v / v^T v after ORC_FSAI_POWER_STEPS steps of the power method
 * (v <- M v / ||M v||_2), M applied as G (A (G^T v)) (never formed), from
 * v_0 with v_0[i] = 2 u_i - 1, u_i = the top 53 bits of splitmix64 draw
 * ((level << 40) + i) of a generator seeded with seed + 1, over 2^53 (the
 * PMIS stream with the next seed).  A Rayleigh quotient never exceeds
 * lambda_max(M), so omega rho(M) >= 4/3; from a random start it comes
 * within a few per cent of it in that many steps, so omega rho(M) stays
 * far below 2.  Products in CSR order from 0.0, dot products in index order.
 */
int orc_fsai_omega(const orc_csr *A, const orc_csr *G, uint64_t seed, int32_t level, double *omega) {
    orc_csr GT = {0, 0, NULL, NULL, NULL};
    int st = orc_transpose(G, &GT);
    const int32_t n = G->nrows;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    double *v = (double *)malloc(sizeof(double) * nn);
    double *t = (double *)malloc(sizeof(double) * nn);
    double *u = (double *)malloc(sizeof(double) * nn);
    double *w = (double *)malloc(sizeof(double) * nn);
    if (!st && (!v || !t || !u || !w)) st = ORC_E_NOMEM;
    if (!st) {
        for (int32_t i = 0; i < n; ++i)
            v[i] = 2.0 * ((double)orc_pmis_rand(seed + 1u, level, i) * 0x1p-53) - 1.0;
        double rq = 0.0;
        for (int k = 0; k < ORC_FSAI_POWER_STEPS; ++k) {
            spmv(&GT, v, t);  /* t = G^T v */
            spmv(A, t, u);    /* u = A G^T v */
            spmv(G, u, w);    /* w = G A G^T v */
            double vv = 0.0, vw = 0.0, ww = 0.0;
            for (int32_t i = 0; i < n; ++i) {
                vv = vv + v[i] * v[i];
                vw = vw + v[i] * w[i];
                ww = ww + w[i] * w[i];
            }
            rq = vw / vv;
            const double s = 1.0 / sqrt(ww);
            for (int32_t i = 0; i < n; ++i) v[i] = w[i] * s;
        }
        *omega = (4.0 / 3.0) / rq;
    }
    free(v); free(t); free(u); free(w);
    orc_csr_free(&GT);
    return st;
}

/* ------------------------------------------------------------------------ */

typedef struct {
    orc_csr A, P, R;
    orc_csr G, GT;           /* FSAI smoother factor and its transpose (FSAI only) */
    uint8_t *strong;
    int32_t *stcnt;
    int8_t *cf;
    double *dinv;
    double omega;
    int32_t rounds;
} orc_level;

#define ORC_MAXLEV 64

struct orc_hier {
    orc_params prm;
    int32_t nlev;            /* levels 0..nlev-1; the last one is solved directly */
    orc_level lev[ORC_MAXLEV];
    double *L;               /* dense Cholesky factor of the last level */
    double *tv;              /* BAMG: test space of the level being built */
};

static int copy_csr(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, orc_csr *o) {
    int32_t nnz = rp[n];
    o->nrows = n; o->ncols = n;
    o->rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    o->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    o->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!o->rp || !o->ci || !o->val) return ORC_E_NOMEM;
    memcpy(o->rp, rp, sizeof(int32_t) * ((size_t)n + 1));
    memcpy(o->ci, ci, sizeof(int32_t) * (size_t)nnz);
    memcpy(o->val, v, sizeof(double) * (size_t)nnz);
    return ORC_OK;
}

void orc_destroy(orc_hier *h) {
    if (!h) return;
    for (int32_t l = 0; l < ORC_MAXLEV; ++l) {
        orc_level *L = &h->lev[l];
        orc_csr_free(&L->A); orc_csr_free(&L->P); orc_csr_free(&L->R);
        orc_csr_free(&L->G); orc_csr_free(&L->GT);
        free(L->strong); free(L->stcnt); free(L->cf); free(L->dinv);
    }
    free(h->L);
    free(h->tv);
    free(h);
}

/*
 * Hierarchy construction, Alg. AMG Set-up, level by level from A_0 = A:
 *   - level l is the last one when n_l <= max_coarse or l = max_levels - 1
 *     (the paper stops where the level is small enough to factorise
 *     directly, read as a size threshold); it is also the last one when
 *     coarsening stalls (no C point, or every point C);
 *   - otherwise: smoother set-up, strength, PMIS, interpolation (direct by
 *     default, or one of the paper's three), R = P^T, A_{l+1} = R (A_l P)
 *     (eq. AcDef);
 *   - the last level is factorised densely (more than 8192 unknowns there
 *     is reported as a stalled coarsening).
 */
int orc_setup(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const orc_params *prm, orc_hier **out) {
    return orc_setup_tv(n, rp, ci, v, 0, NULL, prm, out);
}

/* With BAMG interpolation the level-0 test space is V made orthonormal;
 * level l+1 takes the rows of level l's test space at its C points (P is
 * the identity there). */
int orc_setup_tv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nt, const double *V,
                 const orc_params *prm, orc_hier **out) {
    *out = NULL;
    int st = orc_validate(n, rp, ci, v);
    if (st != ORC_OK) return st;
    int bamg = prm && prm->interp == ORC_INTERP_BAMG;
    if (bamg && (nt < 1 || nt > ORC_MAXNT || !V)) return ORC_E_ARG;
    if (prm && (prm->srqm_iters < 0 || prm->srqm_iters > 100 || (prm->srqm_iters > 0 && !bamg))) return ORC_E_ARG;
    if (prm && prm->smoother == ORC_SMOOTH_AFSAI &&
        (prm->afsai_steps < 0 || prm->afsai_step < 1 ||
         (int64_t)prm->afsai_steps * prm->afsai_step + 1 > ORC_AFSAI_MAXM || !(prm->afsai_eps >= 0.0)))
        return ORC_E_ARG;
    double *TV = NULL;
    if (bamg) {
        TV = (double *)malloc(sizeof(double) * (size_t)n * nt);
        if (!TV) return ORC_E_NOMEM;
        memcpy(TV, V, sizeof(double) * (size_t)n * nt);
        st = orc_orthonormalize(n, nt, TV);
        if (st) { free(TV); return st; }
    }
    orc_hier *h = (orc_hier *)calloc(1, sizeof(orc_hier));
    if (!h) { free(TV); return ORC_E_NOMEM; }
    h->tv = TV;
    if (prm) h->prm = *prm; else orc_params_default(&h->prm);
    if (h->prm.max_levels > ORC_MAXLEV) h->prm.max_levels = ORC_MAXLEV;
    if (h->prm.max_levels < 1) h->prm.max_levels = 1;
    st = copy_csr(n, rp, ci, v, &h->lev[0].A);
    if (st) { orc_destroy(h); return st; }
    int32_t l = 0;
    for (;;) {
        orc_level *L = &h->lev[l];
        int32_t nl = L->A.nrows;
        if (nl <= h->prm.max_coarse || l == h->prm.max_levels - 1) break;
        const int32_t *arp = L->A.rp, *aci = L->A.ci;
        const double *av = L->A.val;
        int32_t nnz = arp[nl];
        L->dinv = (double *)malloc(sizeof(double) * (size_t)nl);
        L->strong = (uint8_t *)malloc((size_t)(nnz > 0 ? nnz : 1));
        L->stcnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)nl);
        L->cf = (int8_t *)malloc((size_t)nl);
        if (!L->dinv || !L->strong || !L->stcnt || !L->cf) { orc_destroy(h); return ORC_E_NOMEM; }
        for (int32_t i = 0; i < nl; ++i) {
            int32_t d = find_in_row(arp, aci, i, i);
            if (d < 0 || !(av[d] > 0.0)) { orc_destroy(h); return ORC_E_NOT_SPD; }
            L->dinv[i] = 1.0 / av[d];
        }
        /* FSAI on this level: always with ORC_SMOOTH_FSAI; with
         * ORC_SMOOTH_FSAI_JACOBI when no row has more than ORC_FSAI_MAXROW
         * entries on or below the diagonal (Jacobi otherwise) */
        int use_fsai = h->prm.smoother == ORC_SMOOTH_FSAI ||
                       (h->prm.smoother == ORC_SMOOTH_FSAI_JACOBI && lower_row_max(&L->A) <= ORC_FSAI_MAXROW);
        if (h->prm.smoother == ORC_SMOOTH_AFSAI) {
            /* adaptive FSAI where every row's candidate set fits, Jacobi otherwise */
            int32_t maxcand = 0;
            st = orc_afsai(&L->A, h->prm.afsai_steps, h->prm.afsai_step, h->prm.afsai_eps, &L->G, &maxcand);
            if (st) { orc_destroy(h); return st; }
            use_fsai = maxcand <= ORC_AFSAI_MAXCAND;
            if (!use_fsai) orc_csr_free(&L->G);
        }
        if (use_fsai) {
            if (h->prm.smoother != ORC_SMOOTH_AFSAI) st = orc_fsai(&L->A, &L->G);
            if (!st) st = orc_transpose(&L->G, &L->GT);
            double w = 0.0;
            if (!st && !(h->prm.omega > 0.0)) st = orc_fsai_omega(&L->A, &L->G, h->prm.seed, l, &w);
            if (st) { orc_destroy(h); return st; }
            L->omega = h->prm.omega > 0.0 ? h->prm.omega : w;
        } else {
            L->omega = h->prm.omega > 0.0 ? h->prm.omega : orc_gershgorin_omega(nl, arp, aci, av);
        }
        if (bamg && l == 0 && h->prm.srqm_iters > 0) {
            /* refine the level-0 test space with the smoother just built,
             * then take an orthonormal basis of it again */
            int32_t done = 0;
            const int fs = L->G.rp != NULL;
            st = orc_srqm(&L->A, L->dinv, fs ? &L->G : NULL, fs ? &L->GT : NULL, nt, TV, h->prm.srqm_iters, &done);
            if (!st) st = orc_orthonormalize(nl, nt, TV);
            if (st) { orc_destroy(h); return st; }
        }
        orc_strength(nl, arp, aci, av, h->prm.theta, L->strong, L->stcnt);
        st = orc_pmis(nl, arp, aci, L->strong, L->stcnt, h->prm.seed, l, L->cf, &L->rounds);
        if (st) { orc_destroy(h); return st; }
        int32_t nc = 0;
        for (int32_t i = 0; i < nl; ++i) if (L->cf[i] == ORC_C) ++nc;
        if (nc == 0 || nc == nl) break;
        if (bamg) {
            st = orc_bamg(nl, arp, aci, L->strong, L->cf, nt, TV, h->prm.bamg_lmin, h->prm.bamg_lmax,
                          h->prm.bamg_eps, h->prm.bamg_mu, &L->P);
            if (!st) {  /* the next level's test space: rows at the C points */
                int32_t c = 0;
                for (int32_t i = 0; i < nl; ++i)
                    if (L->cf[i] == ORC_C) {
                        memmove(TV + (size_t)c * nt, TV + (size_t)i * nt, sizeof(double) * (size_t)nt);
                        ++c;
                    }
            }
        } else {
            st = orc_interp(nl, arp, aci, av, L->strong, L->cf, h->prm.interp, &L->P);
        }
        if (!st && h->prm.psmooth) {  /* one Jacobi step on P with the Jacobi weight of the level */
            double wj = h->prm.omega > 0.0 ? h->prm.omega : orc_gershgorin_omega(nl, arp, aci, av);
            orc_csr Ps = {0, 0, NULL, NULL, NULL};
            st = orc_psmooth(&L->A, L->dinv, wj, &L->P, &Ps);
            if (!st) { orc_csr_free(&L->P); L->P = Ps; }
        }
        if (!st && h->prm.pfilter < 1.0) {  /* filter on the coarse test space (a unit vector without one) */
            int32_t ncl = L->P.ncols;
            double *ones = NULL;
            const double *W = TV;
            int32_t ntw = nt;
            if (!bamg) {
                ones = (double *)malloc(sizeof(double) * (size_t)(ncl > 0 ? ncl : 1));
                if (!ones) { orc_destroy(h); return ORC_E_NOMEM; }
                for (int32_t c = 0; c < ncl; ++c) ones[c] = 1.0;
                W = ones;
                ntw = 1;
            }
            orc_csr Pf = {0, 0, NULL, NULL, NULL};
            st = orc_pfilter(&L->P, h->prm.pfilter, ntw, W, &Pf);
            free(ones);
            if (!st) { orc_csr_free(&L->P); L->P = Pf; }
        }
        if (!st) st = orc_transpose(&L->P, &L->R);
        orc_csr AP = {0, 0, NULL, NULL, NULL};
        if (!st) st = orc_spgemm(&L->A, &L->P, &AP);
        if (!st) st = orc_spgemm(&L->R, &AP, &h->lev[l + 1].A);
        orc_csr_free(&AP);
        if (st) { orc_destroy(h); return st; }
        ++l;
    }
    /* last level: discard any coarsening data computed before a stall */
    orc_level *Lc = &h->lev[l];
    orc_csr_free(&Lc->P); orc_csr_free(&Lc->R); orc_csr_free(&Lc->G); orc_csr_free(&Lc->GT);
    h->nlev = l + 1;
    int32_t nL = Lc->A.nrows;
    if (nL > 8192) { orc_destroy(h); return ORC_E_COARSE; }
    h->L = (double *)calloc((size_t)nL * (size_t)nL, sizeof(double));
    if (!h->L) { orc_destroy(h); return ORC_E_NOMEM; }
    for (int32_t i = 0; i < nL; ++i)
        for (int32_t e = Lc->A.rp[i]; e < Lc->A.rp[i + 1]; ++e)
            h->L[(size_t)i * nL + Lc->A.ci[e]] = Lc->A.val[e];
    if (orc_cholesky(nL, h->L) != 0) { orc_destroy(h); return ORC_E_NOT_SPD; }
    *out = h;
    return ORC_OK;
}

int orc_num_levels(const orc_hier *h) { return h ? h->nlev : 0; }

int orc_level_sizes(const orc_hier *h, int32_t l, int32_t *n, int32_t *nnzA, int32_t *nnzP, int32_t *nc) {
    if (!h || l < 0 || l >= h->nlev) return ORC_E_ARG;
    const orc_level *L = &h->lev[l];
    *n = L->A.nrows;
    *nnzA = L->A.rp[L->A.nrows];
    *nnzP = (l < h->nlev - 1) ? L->P.rp[L->P.nrows] : 0;
    *nc = (l < h->nlev - 1) ? L->P.ncols : 0;
    return ORC_OK;
}

static void copy_out_csr(const orc_csr *m, void *a, void *b, void *c) {
    int32_t nnz = m->rp[m->nrows];
    if (a) memcpy(a, m->rp, sizeof(int32_t) * ((size_t)m->nrows + 1));
    if (b) memcpy(b, m->ci, sizeof(int32_t) * (size_t)nnz);
    if (c) memcpy(c, m->val, sizeof(double) * (size_t)nnz);
}

int orc_export(const orc_hier *h, int32_t l, int32_t what, void *a, void *b, void *c) {
    if (!h || l < 0 || l >= h->nlev) return ORC_E_ARG;
    const orc_level *L = &h->lev[l];
    int last = (l == h->nlev - 1);
    int32_t n = L->A.nrows;
    switch (what) {
    case ORC_X_A: copy_out_csr(&L->A, a, b, c); return ORC_OK;
    case ORC_X_P: if (last) return ORC_E_ARG; copy_out_csr(&L->P, a, b, c); return ORC_OK;
    case ORC_X_R: if (last) return ORC_E_ARG; copy_out_csr(&L->R, a, b, c); return ORC_OK;
    case ORC_X_CF: if (last) return ORC_E_ARG; memcpy(a, L->cf, (size_t)n); return ORC_OK;
    case ORC_X_STRONG: if (last) return ORC_E_ARG; memcpy(a, L->strong, (size_t)L->A.rp[n]); return ORC_OK;
    case ORC_X_DINV: if (last) return ORC_E_ARG; memcpy(a, L->dinv, sizeof(double) * (size_t)n); return ORC_OK;
    case ORC_X_OMEGA: if (last) return ORC_E_ARG; memcpy(a, &L->omega, sizeof(double)); return ORC_OK;
    case ORC_X_STCNT: if (last) return ORC_E_ARG; memcpy(a, L->stcnt, sizeof(int32_t) * (size_t)n); return ORC_OK;
    case ORC_X_ROUNDS: if (last) return ORC_E_ARG; memcpy(a, &L->rounds, sizeof(int32_t)); return ORC_OK;
    case ORC_X_G: if (last || !L->G.rp) return ORC_E_ARG; copy_out_csr(&L->G, a, b, c); return ORC_OK;
    case ORC_X_CHOL: if (!last) return ORC_E_ARG; memcpy(a, h->L, sizeof(double) * (size_t)n * (size_t)n); return ORC_OK;
    default: return ORC_E_ARG;
    }
}

/* t = A s, each row summed in CSR order from 0.0 */
static void spmv(const orc_csr *A, const double *s, double *t) {
    for (int32_t i = 0; i < A->nrows; ++i) {
        double acc = 0.0;
        for (int32_t e = A->rp[i]; e < A->rp[i + 1]; ++e) acc = acc + A->val[e] * s[A->ci[e]];
        t[i] = acc;
    }
}

/*
 * One V-cycle z = M_l y (Alg. AMG application in a V-cycle).  Smoothing is
 * s <- s + omega M^{-1} (y - A s) (eq. smoother) with M = D (Jacobi; the
 * scaled inverse diagonal formed as omega * dinv_i) or M^{-1} = G^T G
 * (FSAI, eq. smo: u = G d, w = G^T u, s_i + omega * w_i).  nu_pre steps from
 * s = 0 (the first of them is s = omega M^{-1} y, since A 0 = 0), residual,
 * restriction by R = P^T, recursion, prolongation and correction, nu_post
 * steps.  On the last level, z = L^{-T} L^{-1} y.
 */
static void smooth_step(const orc_level *L, int fsai, int first, const double *y, double *s, double *t,
                        double *u, double *w) {
    int32_t n = L->A.nrows;
    if (!fsai) {
        if (first) {
            for (int32_t i = 0; i < n; ++i) s[i] = (L->omega * L->dinv[i]) * y[i];
        } else {
            spmv(&L->A, s, t);
            for (int32_t i = 0; i < n; ++i) s[i] = s[i] + (L->omega * L->dinv[i]) * (y[i] - t[i]);
        }
        return;
    }
    if (first) {
        spmv(&L->G, y, u);
        spmv(&L->GT, u, w);
        for (int32_t i = 0; i < n; ++i) s[i] = L->omega * w[i];
    } else {
        spmv(&L->A, s, t);
        for (int32_t i = 0; i < n; ++i) t[i] = y[i] - t[i];
        spmv(&L->G, t, u);
        spmv(&L->GT, u, w);
        for (int32_t i = 0; i < n; ++i) s[i] = s[i] + L->omega * w[i];
    }
}

static void vcycle_level(const orc_hier *h, int32_t l, const double *y, double *z) {
    const orc_level *L = &h->lev[l];
    int32_t n = L->A.nrows;
    if (l == h->nlev - 1) { orc_chol_solve(n, h->L, y, z); return; }
    int32_t nc = L->P.ncols;
    int fsai = L->G.rp != NULL;  /* this level's smoother */
    double *s = z;   /* the smoothed iterate lives in the output */
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *yc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double *dc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    for (int32_t i = 0; i < n; ++i) s[i] = 0.0;
    for (int32_t it = 0; it < h->prm.nu_pre; ++it) smooth_step(L, fsai, it == 0, y, s, t, u, w);
    spmv(&L->A, s, t);
    for (int32_t i = 0; i < n; ++i) t[i] = y[i] - t[i];      /* r = y - A s */
    spmv(&L->R, t, yc);                                       /* y_{l+1} = P^T r */
    vcycle_level(h, l + 1, yc, dc);
    spmv(&L->P, dc, t);                                       /* d_l = P d_{l+1} */
    for (int32_t i = 0; i < n; ++i) s[i] = s[i] + t[i];
    for (int32_t it = 0; it < h->prm.nu_post; ++it) smooth_step(L, fsai, 0, y, s, t, u, w);
    free(t); free(u); free(w); free(yc); free(dc);
}

void orc_vcycle(const orc_hier *h, const double *y, double *z) { vcycle_level(h, 0, y, z); }

static double norm2(int32_t n, const double *x) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s = s + x[i] * x[i];
    return sqrt(s);
}

static double dot(int32_t n, const double *x, const double *y) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s = s + x[i] * y[i];
    return s;
}

/*
 * Preconditioned CG (the paper's Krylov solver, Section 3 LinSolver/PCG),
 * in the standard Hestenes-Stiefel form, started from x_0 = 0 and stopped
 * when the recursively updated residual satisfies ||r_k|| < rtol ||b||
 * (Section 4: the iterative residual's norm smaller than 1e-8 ||b||).
 *   z = M r_k, rho_k = r_k . z, p = z (k = 0) or z + (rho_k / rho_{k-1}) p,
 *   q = A p, sigma = p . q, alpha = rho_k / sigma, x += alpha p, r -= alpha q.
 * sigma <= 0 or rho_k <= 0 is a breakdown.  rtol <= 0 runs exactly
 * max_iter iterations.  hist[k] = ||r_k|| for k <= iters (up to hist_cap).
 * b = 0 returns x = 0 after 0 iterations.
 */
int orc_solve(const orc_hier *h, const double *b, double rtol, int32_t max_iter, int32_t precond,
              double *x, int32_t *iters, double *hist, int32_t hist_cap, double *true_relres) {
    const orc_csr *A = &h->lev[0].A;
    int32_t n = A->nrows;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q) { free(r); free(z); free(p); free(q); return ORC_E_NOMEM; }
    for (int32_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    double bn = norm2(n, b);
    if (hist && hist_cap > 0) hist[0] = bn;
    int status = ORC_OK;
    int32_t k = 0;
    if (bn == 0.0) {
        *iters = 0;
        if (true_relres) *true_relres = 0.0;
        free(r); free(z); free(p); free(q);
        return ORC_OK;
    }
    double rn = bn, rho_old = 0.0;
    for (k = 0;; ++k) {
        if (rtol > 0.0 && rn < rtol * bn) break;
        if (k == max_iter) { status = ORC_MAXIT; break; }
        if (precond) orc_vcycle(h, r, z);
        else for (int32_t i = 0; i < n; ++i) z[i] = r[i];
        double rho = dot(n, r, z);
        if (k == 0) for (int32_t i = 0; i < n; ++i) p[i] = z[i];
        else {
            double beta = rho / rho_old;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        spmv(A, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0) || !(rho > 0.0)) { status = ORC_E_BREAKDOWN; break; }
        double alpha = rho / sigma;
        for (int32_t i = 0; i < n; ++i) { x[i] = x[i] + alpha * p[i]; r[i] = r[i] - alpha * q[i]; }
        rho_old = rho;
        rn = norm2(n, r);
        if (hist && k + 1 < hist_cap) hist[k + 1] = rn;
    }
    *iters = k;
    if (true_relres) {
        spmv(A, x, q);
        for (int32_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
        *true_relres = norm2(n, q) / bn;
    }
    free(r); free(z); free(p); free(q);
    return status;
}
