/*
 * qqa_oracle.c -- plain FP64 CPU reference for the Parallel Quasi-Quantum Annealing
 * (PQQA) replica update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the solver library never links, calls or
 * includes anything from here, and this file includes nothing from the solver.
 *
 * Single-threaded, double precision, no blocking, fusion or reordering: each function
 * spells out one definition of the paper in the paper's order and notation.
 *
 *   S replicas of N relaxed variables, P[i*S + s] = p_i^(s) in [0, 1], row-major with
 *   the replica index contiguous.  Graph: symmetric CSR (row_ptr[n+1] int64,
 *   col[nnz] int32, optional weight[nnz]) or a dense symmetric n x n matrix.
 *
 * Noise and initial values come from a counter-based generator, Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
 * implemented here from that publication.  Stream layout (shared by contract, not by
 * code, with the device implementation):
 *     key     = (seed mod 2^32, seed div 2^32)
 *     counter = (row i, replica quad q, step k, stream)    stream 0 = init, 1 = noise
 *     uniform = ((r >> 8) | 1) * 2^-24                     odd multiples of 2^-24 in (0,1)
 *     normals = Box-Muller (1958) on (u0,u1) and (u2,u3): 4 normals per call
 *
 * Parity status (tests/test_oracle_*.py pin each function against something other
 * than itself):
 *   orc_eval        exact: brute force over every x of small graphs (maximum independent
 *                   sets, maximum cuts, maximum cliques), textbook optima
 *   orc_energy      exact at binary points (equals the discrete objective), closed
 *                   forms at P = 1/2 and for the STD maximiser (appendix proposition)
 *   orc_grad        central finite differences of orc_energy, row sums of the STD term;
 *                   max clique also against the MIS gradient on the complement graph
 *   orc_step        AdamW first-step closed form, projected-gradient fixed point of a
 *                   regular graph (closed-form root), Langevin noise moments
 *   orc_cat_*       categorical K-state variant (graph coloring): K = 2 reduction of the
 *                   entropy to the binary alpha-entropy (appendix proposition), entropy
 *                   extremes, energy at one-hot points = conflict count (brute force),
 *                   central finite differences through the Clamp-normalisation, brute-force
 *                   minimum conflicts and textbook chromatic numbers
 *   orc_philox*     bijectivity (an independent inverse), avalanche, uniform/normal
 *                   goodness-of-fit statistics, distinct streams.  Parity unpinned: the
 *                   generator's published known-answer vectors are not available here, so
 *                   conformance of this implementation of Philox4x32-10 (Salmon et al., SC
 *                   2011) to the published stream is not checked; the GPU's integers are
 *                   compared bit for bit with these.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- problem / step-rule codes ----------------------------------------------------- */
enum { ORC_MIS = 0, ORC_MAXCUT = 1, ORC_MAXCLIQUE = 2 };
enum { ORC_ADAMW = 0, ORC_LANGEVIN = 1 };
enum { ORC_STREAM_INIT = 0, ORC_STREAM_NOISE = 1 };

typedef struct {
    double gamma_min, gamma_max; /* entropy coefficient, linear schedule (Implementation; App. Annealing Schedule) */
    double lr;                   /* eta, step size (Eq. 11; App. Configuration of Optimizer) */
    double weight_decay;         /* AdamW decoupled decay */
    double temperature;          /* T in sqrt(2 eta T) xi (Eq. 11) */
    double comm_alpha;           /* alpha of the STD communication term (Eq. 10) */
    int32_t entropy_alpha;       /* alpha of the alpha-entropy (Eq. 7), even */
    int32_t rule;                /* ORC_ADAMW or ORC_LANGEVIN */
    double beta1, beta2, adam_eps;
    double lambda;               /* MIS / max-clique penalty coefficient */
    int32_t problem;             /* ORC_MIS, ORC_MAXCUT or ORC_MAXCLIQUE */
    int32_t pad_;
} orc_params;

typedef struct {
    int32_t n;
    int32_t dense;          /* 1: W is n*n row-major, CSR fields unused */
    const int64_t *row_ptr; /* n+1 */
    const int32_t *col;     /* nnz */
    const double *weight;   /* nnz or NULL (all ones) */
    const double *W;        /* n*n when dense */
} orc_graph;

/* ---- Philox4x32-10 ------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u; /* round multipliers */
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u; /* key schedule increments */

/* One Philox4x32 round: two 32x32->64 multiplies act as S-boxes, the key is xor-ed
   into the high halves and the words are permuted. */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t o0 = hi1 ^ c[1] ^ k[0];
    uint32_t o2 = hi0 ^ c[3] ^ k[1];
    c[0] = o0; c[1] = lo1; c[2] = o2; c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += PHILOX_W0; k[1] += PHILOX_W1; }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* Inverse of the 10-round map, used by the tests to show the map is a bijection. */
void orc_philox4x32_10_inverse(const uint32_t out[4], const uint32_t key[2], uint32_t ctr[4]) {
    uint32_t ks[10][2];
    ks[0][0] = key[0]; ks[0][1] = key[1];
    for (int r = 1; r < 10; ++r) { ks[r][0] = ks[r-1][0] + PHILOX_W0; ks[r][1] = ks[r-1][1] + PHILOX_W1; }
    uint32_t c[4] = {out[0], out[1], out[2], out[3]};
    for (int r = 9; r >= 0; --r) {
        /* forward: c' = (hi1^c1^k0, lo1, hi0^c3^k1, lo0) with (hi0,lo0)=M0*c0, (hi1,lo1)=M1*c2.
           lo0 and lo1 determine c0 and c2 because the multipliers are odd. */
        uint32_t lo1 = c[1], lo0 = c[3];
        /* modular inverse of an odd 32-bit multiplier by Newton iteration */
        uint32_t inv0 = PHILOX_M0, inv1 = PHILOX_M1;
        for (int it = 0; it < 5; ++it) { inv0 *= 2u - PHILOX_M0 * inv0; inv1 *= 2u - PHILOX_M1 * inv1; }
        uint32_t c0 = lo0 * inv0, c2 = lo1 * inv1;
        uint32_t hi0 = (uint32_t)(((uint64_t)PHILOX_M0 * c0) >> 32);
        uint32_t hi1 = (uint32_t)(((uint64_t)PHILOX_M1 * c2) >> 32);
        uint32_t c1 = c[0] ^ hi1 ^ ks[r][0];
        uint32_t c3 = c[2] ^ hi0 ^ ks[r][1];
        c[0] = c0; c[1] = c1; c[2] = c2; c[3] = c3;
    }
    memcpy(ctr, c, sizeof c);
}

static void philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 24-bit uniform on (0,1): odd multiples of 2^-24, exactly representable in binary32. */
double orc_u01(uint32_t r) { return (double)((r >> 8) | 1u) * (1.0 / 16777216.0); }

/* Box-Muller: (u0,u1) -> (R cos t, R sin t), R = sqrt(-2 ln u0), t = 2 pi u1; same for (u2,u3). */
void orc_normals4(const uint32_t r[4], double xi[4]) {
    const double two_pi = 6.283185307179586476925286766559;
    double ua = orc_u01(r[0]), ub = orc_u01(r[1]), uc = orc_u01(r[2]), ud = orc_u01(r[3]);
    double R1 = sqrt(-2.0 * log(ua)), R2 = sqrt(-2.0 * log(uc));
    xi[0] = R1 * cos(two_pi * ub);
    xi[1] = R1 * sin(two_pi * ub);
    xi[2] = R2 * cos(two_pi * ud);
    xi[3] = R2 * sin(two_pi * ud);
}

/* Raw integers of the stream for rows [0,n), quads [0,nquads): out[(i*nquads + q)*4 + j]. */
void orc_philox_grid(uint64_t seed, int32_t n, int32_t nquads, uint32_t k, uint32_t stream, uint32_t *out) {
    for (int32_t i = 0; i < n; ++i)
        for (int32_t q = 0; q < nquads; ++q)
            philox_seeded(seed, (uint32_t)i, (uint32_t)q, k, stream, out + ((size_t)i * nquads + q) * 4);
}

/* Gaussian noise xi (n x S) of step k: replica s takes normal (s mod 4) of quad s/4. */
void orc_noise(uint64_t seed, int32_t n, int32_t S, uint32_t k, double *xi) {
    for (int32_t i = 0; i < n; ++i)
        for (int32_t q = 0; 4 * q < S; ++q) {
            uint32_t r[4]; double z[4];
            philox_seeded(seed, (uint32_t)i, (uint32_t)q, k, ORC_STREAM_NOISE, r);
            orc_normals4(r, z);
            for (int j = 0; j < 4 && 4 * q + j < S; ++j) xi[(size_t)i * S + 4 * q + j] = z[j];
        }
}

/* Initial relaxed variables: p ~ U(0,1) per replica (the paper does not fix the start). */
void orc_init(uint64_t seed, int32_t n, int32_t S, double *P) {
    for (int32_t i = 0; i < n; ++i)
        for (int32_t q = 0; 4 * q < S; ++q) {
            uint32_t r[4];
            philox_seeded(seed, (uint32_t)i, (uint32_t)q, 0u, ORC_STREAM_INIT, r);
            for (int j = 0; j < 4 && 4 * q + j < S; ++j) P[(size_t)i * S + 4 * q + j] = orc_u01(r[j]);
        }
}

/* ---- schedule ------------------------------------------------------------------------ */
/* gamma increases linearly from gamma_min (first update) to gamma_max (last update). */
double orc_gamma(const orc_params *pr, int32_t t, int32_t K) {
    if (K <= 1) return pr->gamma_min;
    return pr->gamma_min + (pr->gamma_max - pr->gamma_min) * (double)t / (double)(K - 1);
}

static double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

static double edge_weight(const orc_graph *g, int64_t e) { return g->weight ? g->weight[e] : 1.0; }

/* ---- energy (for finite differences and closed-form pins) ----------------------------- */
/* p^T A p of replica s (each ordered pair (i, j) with A_ij != 0 once) */
static double quad_form(const orc_graph *g, int32_t S, const double *P, int32_t s) {
    const int32_t n = g->n;
    double quad = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double pi = P[(size_t)i * S + s];
        if (g->dense) {
            for (int32_t j = 0; j < n; ++j) quad += pi * g->W[(size_t)i * n + j] * P[(size_t)j * S + s];
        } else {
            for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e)
                quad += pi * edge_weight(g, e) * P[(size_t)g->col[e] * S + s];
        }
    }
    return quad;
}

/* 1^T p of replica s */
static double column_sum(int32_t n, int32_t S, const double *P, int32_t s) {
    double t = 0.0;
    for (int32_t i = 0; i < n; ++i) t += P[(size_t)i * S + s];
    return t;
}

/* Relaxed objective l^(p) of one replica (continuous relaxation of the penalised loss,
   energies of the appendix "Energy Function of Benchmark Problems"):
     MIS:       -sum_i p_i + lambda * p^T A p / 2          (c = 1)
     MaxCut:    -sum_{(i,j) in E} A_ij (1 - (2p_i - 1)(2p_j - 1)) / 2
     MaxClique: -sum_i p_i + lambda/2 * ( 1^T p (1^T p - 1) - p^T A p )   (c = 1)          */
static double relaxed_objective(const orc_params *pr, const orc_graph *g, int32_t S, const double *P, int32_t s) {
    const int32_t n = g->n;
    double l = 0.0;
    if (pr->problem == ORC_MAXCLIQUE) {
        const double T = column_sum(n, S, P, s);
        return -T + pr->lambda / 2.0 * (T * (T - 1.0) - quad_form(g, S, P, s));
    }
    if (pr->problem == ORC_MIS) {
        double quad = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            double pi = P[(size_t)i * S + s];
            l -= pi;
            if (g->dense) {
                for (int32_t j = 0; j < n; ++j) quad += pi * g->W[(size_t)i * n + j] * P[(size_t)j * S + s];
            } else {
                for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e)
                    quad += pi * edge_weight(g, e) * P[(size_t)g->col[e] * S + s];
            }
        }
        l += pr->lambda * quad / 2.0;
    } else {
        for (int32_t i = 0; i < n; ++i) {
            double zi = 2.0 * P[(size_t)i * S + s] - 1.0;
            if (g->dense) {
                for (int32_t j = i + 1; j < n; ++j) {
                    double zj = 2.0 * P[(size_t)j * S + s] - 1.0;
                    l -= g->W[(size_t)i * n + j] * (1.0 - zi * zj) / 2.0;
                }
            } else {
                for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                    int32_t j = g->col[e];
                    if (j <= i) continue; /* each undirected edge once */
                    double zj = 2.0 * P[(size_t)j * S + s] - 1.0;
                    l -= edge_weight(g, e) * (1.0 - zi * zj) / 2.0;
                }
            }
        }
    }
    return l;
}

/* alpha-entropy s(p) = sum_i {1 - (2 p_i - 1)^alpha}   (Eq. 7) */
static double alpha_entropy(int alpha, int32_t n, int32_t S, const double *P, int32_t s) {
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) acc += 1.0 - ipow(2.0 * P[(size_t)i * S + s] - 1.0, alpha);
    return acc;
}

/* empirical (population) standard deviation over the S replicas of variable i (Eq. 10) */
static double replica_std(int32_t S, const double *row) {
    double mu = 0.0;
    for (int32_t s = 0; s < S; ++s) mu += row[s];
    mu /= (double)S;
    double var = 0.0;
    for (int32_t s = 0; s < S; ++s) var += (row[s] - mu) * (row[s] - mu);
    return sqrt(var / (double)S);
}

/* R^ = sum_s [ l^(p^(s)) + gamma s(p^(s)) ] - S alpha_c sum_i STD_s[p_i^(s)]   (Eqs. 6, 10) */
double orc_energy(const orc_params *pr, const orc_graph *g, int32_t S, const double *P, double gamma) {
    double R = 0.0;
    for (int32_t s = 0; s < S; ++s)
        R += relaxed_objective(pr, g, S, P, s) + gamma * alpha_entropy(pr->entropy_alpha, g->n, S, P, s);
    double stdsum = 0.0;
    for (int32_t i = 0; i < g->n; ++i) stdsum += replica_std(S, P + (size_t)i * S);
    return R - (double)S * pr->comm_alpha * stdsum;
}

/* ---- gradient of R^ with respect to P -------------------------------------------------- */
/* gf: gradient of the relaxed objective
         MIS        -1 + lambda * sum_j A_ij p_j
         MaxCut     sum_j A_ij (2 p_j - 1)
         MaxClique  -1 + lambda * (1^T p - 1/2 - sum_j A_ij p_j)   (1^T p over the replica's column)
   ge: gradient of gamma s(p): -2 alpha gamma (2p - 1)^(alpha - 1)
   gc: gradient of -S alpha_c STD_i: -alpha_c (p - mu_i) / sigma_i, taken as 0 when sigma_i = 0
   sigma (optional, n): sigma_i                                                            */
void orc_grad(const orc_params *pr, const orc_graph *g, int32_t S, const double *P, double gamma,
              double *gf, double *ge, double *gc, double *sigma) {
    const int32_t n = g->n;
    const int maxcut = pr->problem == ORC_MAXCUT;
    double *colsum = (double *)malloc((size_t)(S > 0 ? S : 1) * sizeof(double));
    for (int32_t s = 0; s < S; ++s) colsum[s] = column_sum(n, S, P, s);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t s = 0; s < S; ++s) {
            double c = 0.0;
            if (g->dense) {
                for (int32_t j = 0; j < n; ++j) {
                    double pj = P[(size_t)j * S + s];
                    c += g->W[(size_t)i * n + j] * (maxcut ? 2.0 * pj - 1.0 : pj);
                }
            } else {
                for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                    double pj = P[(size_t)g->col[e] * S + s];
                    c += edge_weight(g, e) * (maxcut ? 2.0 * pj - 1.0 : pj);
                }
            }
            if (pr->problem == ORC_MIS) gf[(size_t)i * S + s] = -1.0 + pr->lambda * c;
            else if (maxcut) gf[(size_t)i * S + s] = c;
            else gf[(size_t)i * S + s] = -1.0 + pr->lambda * (colsum[s] - 0.5 - c);
            double z = 2.0 * P[(size_t)i * S + s] - 1.0;
            ge[(size_t)i * S + s] = -2.0 * (double)pr->entropy_alpha * gamma * ipow(z, pr->entropy_alpha - 1);
        }
        const double *row = P + (size_t)i * S;
        double mu = 0.0;
        for (int32_t s = 0; s < S; ++s) mu += row[s];
        mu /= (double)S;
        double sd = replica_std(S, row);
        if (sigma) sigma[i] = sd;
        for (int32_t s = 0; s < S; ++s)
            gc[(size_t)i * S + s] = sd > 0.0 ? -pr->comm_alpha * (row[s] - mu) / sd : 0.0;
    }
    free(colsum);
}

/* Sum of the magnitudes of every term that makes up the objective gradient gf of replica
   s at variable i: 1 + lambda sum_j |A_ij p_j| (MIS), sum_j |A_ij (2 p_j - 1)| (max-cut),
   1 + lambda (sum_j |p_j| + 1/2 + sum_j |A_ij p_j|) (max clique).
   A diagnostic for comparisons: it sets the scale of the rounding error of any
   finite-precision evaluation of gf. */
static double objective_term_magnitude(const orc_params *pr, const orc_graph *g, int32_t S, const double *P,
                                       int32_t i, int32_t s) {
    const int32_t n = g->n;
    double acc = pr->problem == ORC_MAXCUT ? 0.0 : 1.0;
    const double scale = pr->problem == ORC_MAXCUT ? 1.0 : pr->lambda;
    if (pr->problem == ORC_MAXCLIQUE) {
        for (int32_t j = 0; j < n; ++j) acc += scale * fabs(P[(size_t)j * S + s]);
        acc += scale * 0.5;
    }
    if (g->dense) {
        for (int32_t j = 0; j < n; ++j) {
            double pj = P[(size_t)j * S + s];
            acc += scale * fabs(g->W[(size_t)i * n + j] * (pr->problem == ORC_MAXCUT ? 2.0 * pj - 1.0 : pj));
        }
    } else {
        for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
            double pj = P[(size_t)g->col[e] * S + s];
            acc += scale * fabs(edge_weight(g, e) * (pr->problem == ORC_MAXCUT ? 2.0 * pj - 1.0 : pj));
        }
    }
    return acc;
}

static double p_row_in(const double *P, int32_t S, size_t e) { (void)S; return P[e]; }

/* ---- one update (Sensitive Transitions, Eq. 11, with AdamW in place of the plain step) ---
   t is the 0-based update index (AdamW step count k = t + 1), K the schedule length.
   Optional diagnostics (n*S): pre_clamp = value before the clamp, gsum = g,
   gabs = magnitude of all terms of g before cancellation: those of gf, |ge|, and
   alpha_c (|p| + |mu_i|) / sigma_i for gc;  sigma (n).                                     */
void orc_step(const orc_params *pr, const orc_graph *g, int32_t S, int32_t t, int32_t K, uint64_t seed,
              const double *P_in, double *P_out, double *m, double *v,
              double *pre_clamp, double *gsum, double *gabs, double *sigma) {
    const int32_t n = g->n;
    const size_t NS = (size_t)n * S;
    const double gamma = orc_gamma(pr, t, K);
    const uint32_t k = (uint32_t)t + 1u;
    double *gf = (double *)malloc(NS * sizeof(double));
    double *ge = (double *)malloc(NS * sizeof(double));
    double *gc = (double *)malloc(NS * sizeof(double));
    double *xi = (double *)malloc(NS * sizeof(double));
    double *sigma_row = (double *)malloc((size_t)n * sizeof(double));
    double *mu_row = (double *)malloc((size_t)n * sizeof(double));
    orc_grad(pr, g, S, P_in, gamma, gf, ge, gc, sigma_row);
    if (sigma) memcpy(sigma, sigma_row, (size_t)n * sizeof(double));
    for (int32_t i = 0; i < n; ++i) {
        double mu = 0.0;
        for (int32_t s = 0; s < S; ++s) mu += P_in[(size_t)i * S + s];
        mu_row[i] = mu / (double)S;
    }
    orc_noise(seed, n, S, k, xi);
    const double bc1 = 1.0 - pow(pr->beta1, (double)k);
    const double bc2 = 1.0 - pow(pr->beta2, (double)k);
    const double noise_scale = sqrt(2.0 * pr->lr * pr->temperature);
    for (size_t e = 0; e < NS; ++e) {
        double grad = gf[e] + ge[e] + gc[e];
        double p = P_in[e];
        if (pr->rule == ORC_ADAMW) {
            /* AdamW (Loshchilov & Hutter): decoupled decay, moment updates, bias correction */
            p = p - pr->lr * pr->weight_decay * p;
            m[e] = pr->beta1 * m[e] + (1.0 - pr->beta1) * grad;
            v[e] = pr->beta2 * v[e] + (1.0 - pr->beta2) * grad * grad;
            double mhat = m[e] / bc1, vhat = v[e] / bc2;
            p = p - pr->lr * mhat / (sqrt(vhat) + pr->adam_eps);
        } else {
            p = p - pr->lr * grad; /* plain gradient step of Eq. 11 */
        }
        p = p + noise_scale * xi[e]; /* sqrt(2 eta T) xi */
        if (pre_clamp) pre_clamp[e] = p;
        if (gsum) gsum[e] = grad;
        if (gabs) {
            const int32_t i = (int32_t)(e / (size_t)S);
            double comm = 0.0;
            if (sigma_row[i] > 0.0) comm = pr->comm_alpha * (fabs(p_row_in(P_in, S, e)) + fabs(mu_row[i])) / sigma_row[i];
            gabs[e] = objective_term_magnitude(pr, g, S, P_in, i, (int32_t)(e % (size_t)S)) + fabs(ge[e]) + comm;
        }
        P_out[e] = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p); /* sigma = Clamp to [0,1] */
    }
    free(gf); free(ge); free(gc); free(xi); free(sigma_row); free(mu_row);
}

/* Updates t0 .. t1-1 of a K-update schedule applied in place to (P, m, v). */
void orc_run(const orc_params *pr, const orc_graph *g, int32_t S, int32_t t0, int32_t t1, int32_t K,
             uint64_t seed, double *P, double *m, double *v) {
    const size_t NS = (size_t)g->n * S;
    double *tmp = (double *)malloc(NS * sizeof(double));
    for (int32_t t = t0; t < t1; ++t) {
        orc_step(pr, g, S, t, K, seed, P, tmp, m, v, NULL, NULL, NULL, NULL);
        memcpy(P, tmp, NS * sizeof(double));
    }
    free(tmp);
}

/* ---- rounding and exact evaluation ------------------------------------------------------
   x_i = Theta(p_i - 1/2) with Theta(0) = 0, i.e. x = [p > 1/2].
   MIS:    size = sum_i x_i, viol = #{(i,j) in E : x_i = x_j = 1}, l = -size + lambda*viol
   MaxCut: cut  = sum_{(i,j) in E} w_ij [x_i != x_j] counted in units of 2^-16, l = -cut
   MaxClique: size = sum_i x_i, viol = #{i < j : x_i = x_j = 1, (i,j) not in E}
           = size (size - 1) / 2 - #{(i,j) in E : x_i = x_j = 1},  l = -size + lambda*viol
           (the appendix energy at binary x: its bracket counts each such pair twice)
   Integer arithmetic throughout; weights must be integer multiples of 2^-16.
   best = replica minimising (viol > 0, l, s) lexicographically.  Returns 0, or -1 if a
   weight is off the 2^-16 grid.                                                          */
int orc_eval(int32_t problem, int64_t lambda, const orc_graph *g, int32_t S, const double *P,
             int64_t *size_or_cut, int64_t *viol, int64_t *obj, int32_t *best) {
    const int32_t n = g->n;
    for (int32_t s = 0; s < S; ++s) {
        int64_t a = 0, b = 0;
        const int counts = problem == ORC_MIS || problem == ORC_MAXCLIQUE;
        for (int32_t i = 0; i < n; ++i) {
            int xi = P[(size_t)i * S + s] > 0.5;
            if (counts) a += xi;
            int32_t deg = g->dense ? n : (int32_t)(g->row_ptr[i + 1] - g->row_ptr[i]);
            for (int32_t u = 0; u < deg; ++u) {
                int32_t j; double w;
                if (g->dense) { j = u; w = g->W[(size_t)i * n + j]; }
                else { int64_t e = g->row_ptr[i] + u; j = g->col[e]; w = edge_weight(g, e); }
                if (j <= i || w == 0.0) continue;
                int xj = P[(size_t)j * S + s] > 0.5;
                if (counts) {
                    b += (xi && xj);
                } else {
                    double qd = w * 65536.0;
                    int64_t q = (int64_t)llround(qd);
                    if ((double)q != qd) return -1;
                    if (xi != xj) a += q;
                }
            }
        }
        size_or_cut[s] = a;
        if (problem == ORC_MAXCLIQUE) b = a * (a - 1) / 2 - b; /* selected pairs that are not edges */
        viol[s] = counts ? b : 0;
        obj[s] = counts ? -a + lambda * b : -a;
    }
    int32_t bi = 0;
    for (int32_t s = 1; s < S; ++s) {
        int fs = viol[s] > 0, fb = viol[bi] > 0;
        if (fs < fb || (fs == fb && obj[s] < obj[bi])) bi = s;
    }
    *best = bi;
    return 0;
}


/* =====================================================================================
 * Categorical K-state QQA (appendix "Generalization to discrete optimization problems" and
 * "Transformation for general discrete variables"), for graph coloring.
 *
 * State per replica s: V in [0,1]^{N x K}, stored V[((i*K + k) * S) + s] (the (i, k) pairs
 * as rows, replicas contiguous).  Probabilities sigma_ik = V_ik / Z_i, Z_i = sum_k V_ik
 * (Clamp-normalisation; V is kept clamped, as p is in the binary method); a row with
 * Z_i = 0 reads as uniform, sigma_ik = 1/K, with Z_i taken as 1 in the chain rule.
 *
 *   l(sigma)   = sum_{(i,j) in E, i<j} sum_k sigma_ik sigma_jk     (expected conflicts)
 *   s_K(sigma) = sum_i { 1 - c sum_k (K sigma_ik - 1)^alpha },  c = 1 / ((K-1)((K-1)^(alpha-1) + 1))
 *   R          = sum_s [ l + gamma s_K ] - S alpha_c sum_{i,k} STD_s[sigma_ik]
 * g = dR/dsigma per element, and dR/dV_ik = (g_ik - sum_k' sigma_ik' g_ik') / Z_i.
 * The update is the binary method's: AdamW on V with that gradient, + sqrt(2 eta T) xi,
 * Clamp to [0,1].  Noise and start use the Philox stream with row index i*K + k.
 * Rounding: x_i = argmax_k V_ik (first maximum); cost = #{(i,j) in E : x_i = x_j}.
 * ===================================================================================== */

static size_t cat_at(int32_t K, int32_t S, int32_t i, int32_t k, int32_t s) {
    return ((size_t)i * K + k) * S + s;
}

/* sigma from V, and Z (n*S, with 0 kept as 0) */
void orc_cat_sigma(int32_t n, int32_t K, int32_t S, const double *V, double *sigma, double *Z) {
    for (int32_t i = 0; i < n; ++i)
        for (int32_t s = 0; s < S; ++s) {
            double z = 0.0;
            for (int32_t k = 0; k < K; ++k) z += V[cat_at(K, S, i, k, s)];
            if (Z) Z[(size_t)i * S + s] = z;
            for (int32_t k = 0; k < K; ++k)
                sigma[cat_at(K, S, i, k, s)] = z > 0.0 ? V[cat_at(K, S, i, k, s)] / z : 1.0 / (double)K;
        }
}

static double cat_entropy_coef(int32_t K, int alpha) {
    return 1.0 / ((double)(K - 1) * (ipow((double)(K - 1), alpha - 1) + 1.0));
}

/* s_K of one replica's sigma */
double orc_cat_entropy(int32_t n, int32_t K, int32_t S, int alpha, const double *sigma, int32_t s) {
    const double c = cat_entropy_coef(K, alpha);
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double t = 0.0;
        for (int32_t k = 0; k < K; ++k) t += ipow((double)K * sigma[cat_at(K, S, i, k, s)] - 1.0, alpha);
        acc += 1.0 - c * t;
    }
    return acc;
}

/* R of the categorical model (graph coloring objective) */
double orc_cat_energy(const orc_params *pr, const orc_graph *g, int32_t K, int32_t S, const double *V, double gamma) {
    const int32_t n = g->n;
    const size_t NKS = (size_t)n * K * S;
    double *sg = (double *)malloc(NKS * sizeof(double));
    orc_cat_sigma(n, K, S, V, sg, NULL);
    double R = 0.0;
    for (int32_t s = 0; s < S; ++s) {
        double l = 0.0;
        for (int32_t i = 0; i < n; ++i)
            for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                const int32_t j = g->col[e];
                if (j <= i) continue;
                for (int32_t k = 0; k < K; ++k) l += sg[cat_at(K, S, i, k, s)] * sg[cat_at(K, S, j, k, s)];
            }
        R += l + gamma * orc_cat_entropy(n, K, S, pr->entropy_alpha, sg, s);
    }
    double stdsum = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < K; ++k) stdsum += replica_std(S, sg + cat_at(K, S, i, k, 0));
    free(sg);
    return R - (double)S * pr->comm_alpha * stdsum;
}

/* dR/dV (n*K*S); optional gabs = magnitude of every term of dR/dV before cancellation:
   (a_ik + sum_k' sigma_ik' a_ik') / Z with a_ik = sum_j |sigma_jk| + |entropy term|
   + alpha_c (|sigma| + |mu|) / std. */
void orc_cat_grad(const orc_params *pr, const orc_graph *g, int32_t K, int32_t S, const double *V, double gamma,
                  double *gV, double *gabs) {
    const int32_t n = g->n;
    const size_t NKS = (size_t)n * K * S;
    double *sg = (double *)malloc(NKS * sizeof(double));
    double *Z = (double *)malloc((size_t)n * S * sizeof(double));
    double *G = (double *)malloc(NKS * sizeof(double));
    double *A = (double *)malloc(NKS * sizeof(double));
    orc_cat_sigma(n, K, S, V, sg, Z);
    const double c = cat_entropy_coef(K, pr->entropy_alpha);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < K; ++k) {
            const double *row = sg + cat_at(K, S, i, k, 0);
            double mu = 0.0;
            for (int32_t s = 0; s < S; ++s) mu += row[s];
            mu /= (double)S;
            const double sd = replica_std(S, row);
            for (int32_t s = 0; s < S; ++s) {
                double cpl = 0.0, cabs = 0.0;
                for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                    const double x = sg[cat_at(K, S, g->col[e], k, s)];
                    cpl += x;
                    cabs += fabs(x);
                }
                const double z = (double)K * row[s] - 1.0;
                const double ent = -gamma * c * (double)pr->entropy_alpha * (double)K * ipow(z, pr->entropy_alpha - 1);
                const double com = sd > 0.0 ? -pr->comm_alpha * (row[s] - mu) / sd : 0.0;
                G[cat_at(K, S, i, k, s)] = cpl + ent + com;
                A[cat_at(K, S, i, k, s)] = cabs + fabs(ent) + (sd > 0.0 ? pr->comm_alpha * (fabs(row[s]) + fabs(mu)) / sd : 0.0);
            }
        }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t s = 0; s < S; ++s) {
            double d = 0.0, da = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                d += sg[cat_at(K, S, i, k, s)] * G[cat_at(K, S, i, k, s)];
                da += sg[cat_at(K, S, i, k, s)] * A[cat_at(K, S, i, k, s)];
            }
            const double z = Z[(size_t)i * S + s] > 0.0 ? Z[(size_t)i * S + s] : 1.0;
            for (int32_t k = 0; k < K; ++k) {
                gV[cat_at(K, S, i, k, s)] = (G[cat_at(K, S, i, k, s)] - d) / z;
                if (gabs) gabs[cat_at(K, S, i, k, s)] = (A[cat_at(K, S, i, k, s)] + da) / z;
            }
        }
    free(sg); free(Z); free(G); free(A);
}

/* One categorical update t of a Kt-update schedule (same step rule as orc_step). */
void orc_cat_step(const orc_params *pr, const orc_graph *g, int32_t K, int32_t S, int32_t t, int32_t Kt,
                  uint64_t seed, const double *V_in, double *V_out, double *m, double *v,
                  double *pre_clamp, double *gsum, double *gabs) {
    const int32_t n = g->n;
    const size_t NKS = (size_t)n * K * S;
    const double gamma = orc_gamma(pr, t, Kt);
    const uint32_t kk = (uint32_t)t + 1u;
    double *gV = (double *)malloc(NKS * sizeof(double));
    double *xi = (double *)malloc(NKS * sizeof(double));
    orc_cat_grad(pr, g, K, S, V_in, gamma, gV, gabs);
    orc_noise(seed, n * K, S, kk, xi); /* row index i*K + k */
    const double bc1 = 1.0 - pow(pr->beta1, (double)kk);
    const double bc2 = 1.0 - pow(pr->beta2, (double)kk);
    const double noise_scale = sqrt(2.0 * pr->lr * pr->temperature);
    for (size_t e = 0; e < NKS; ++e) {
        const double grad = gV[e];
        double p = V_in[e];
        if (pr->rule == ORC_ADAMW) {
            p = p - pr->lr * pr->weight_decay * p;
            m[e] = pr->beta1 * m[e] + (1.0 - pr->beta1) * grad;
            v[e] = pr->beta2 * v[e] + (1.0 - pr->beta2) * grad * grad;
            p = p - pr->lr * (m[e] / bc1) / (sqrt(v[e] / bc2) + pr->adam_eps);
        } else {
            p = p - pr->lr * grad;
        }
        p = p + noise_scale * xi[e];
        if (pre_clamp) pre_clamp[e] = p;
        if (gsum) gsum[e] = grad;
        V_out[e] = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
    }
    free(gV); free(xi);
}

void orc_cat_run(const orc_params *pr, const orc_graph *g, int32_t K, int32_t S, int32_t t0, int32_t t1, int32_t Kt,
                 uint64_t seed, double *V, double *m, double *v) {
    const size_t NKS = (size_t)g->n * K * S;
    double *tmp = (double *)malloc(NKS * sizeof(double));
    for (int32_t t = t0; t < t1; ++t) {
        orc_cat_step(pr, g, K, S, t, Kt, seed, V, tmp, m, v, NULL, NULL, NULL);
        memcpy(V, tmp, NKS * sizeof(double));
    }
    free(tmp);
}

/* Rounding and exact cost: colors[n*S] (x_i per replica), conflicts[S]; best = replica with
   the fewest conflicts (lowest index among ties). */
void orc_cat_eval(const orc_graph *g, int32_t K, int32_t S, const double *V, int32_t *colors, int64_t *conflicts,
                  int32_t *best) {
    const int32_t n = g->n;
    for (int32_t s = 0; s < S; ++s) {
        for (int32_t i = 0; i < n; ++i) {
            int32_t arg = 0;
            for (int32_t k = 1; k < K; ++k)
                if (V[cat_at(K, S, i, k, s)] > V[cat_at(K, S, i, arg, s)]) arg = k;
            colors[(size_t)i * S + s] = arg;
        }
        int64_t c = 0;
        for (int32_t i = 0; i < n; ++i)
            for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                const int32_t j = g->col[e];
                if (j > i && colors[(size_t)i * S + s] == colors[(size_t)j * S + s]) ++c;
            }
        conflicts[s] = c;
    }
    int32_t b = 0;
    for (int32_t s = 1; s < S; ++s)
        if (conflicts[s] < conflicts[b]) b = s;
    *best = b;
}
