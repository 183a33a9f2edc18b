/*
 * CPU oracle for two-dimensional parallel tempering (2D-PT).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, sequential, slow
 * reference that the GPU library is checked against.  Nothing in the library
 * links, includes or calls it; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the GPU
 * path: its random generator, colour ranks, energies, swap rules and
 * schedule are all written out here from the paper and from the published
 * definition of the generator.
 *
 * What it computes (paper references are by section / equation / algorithm):
 *   - energy of a replica in penalty column j: E_j = f + P_j g   (Eq. 1)
 *     with f = -sum_{i<j} J_ij s_i s_j - sum_i b_i s_i and either
 *     g = sum over copy edges of (s_a - s_b)^2  (section on graph
 *     sparsification with copy constraints; 4 per violated edge in +-1 form)
 *     or, for general constraints (Eq. 1 only asks g >= 0 with g = 0 exactly
 *     on feasible states), a sum of squared integer linear forms
 *     g = sum_t (sum_{i in t} a_ti s_i + d_t)^2: an equality constraint
 *     sum_i w_i x_i = c on bits x = (1 + s) / 2 is the form a = w,
 *     d = sum_i w_i - 2 c (g = 4 (w.x - c)^2); one-hot groups and inequality
 *     constraints with slack spins, which the introduction names, are of
 *     this kind, and a copy edge is a = (1, -1), d = 0
 *   - Monte Carlo sweeps: heat-bath single-spin updates visiting colour
 *     classes in ascending order, P(s_i = +1) = sigma(2 beta h_i) with
 *     h_i = sum_j J_ij s_j + b_i + P c_i, where -s_i c_i collects the terms
 *     of g that depend on s_i: c_i = 2 sum_{copies k of i} s_k for copy
 *     edges (the ferromagnetic coupling 2P that P (s_a - s_b)^2 amounts
 *     to), and c_i = -2 sum_{t ni i} a_ti (r_t - a_ti s_i) with
 *     r_t = sum_{j in t} a_tj s_j + d_t for general constraints
 *     (Algorithm 1 only says "perform sweeps"; heat-bath is the reading
 *     adopted)
 *   - P-swaps along a row: accept with min(1, exp(beta dP dg))    (Eq. 2)
 *   - beta-swaps along a column: accept with min(1, exp(dbeta dE)) (Eq. 3)
 *     (both are the axis cases of the two-replica rule of Appendix A)
 *   - the round structure of Algorithm 1: every replica sweeps, E and g are
 *     taken from the final state, then one swap direction with alternating
 *     even/odd pairs, the direction flipping after every even round; the
 *     bottom-right replica (largest beta, largest P) is recorded.
 *
 * Fixed-point: couplings, fields and penalties are Q12 integers, so h, f,
 * g, dE and dP*dg are exact integers.  The two decisions that need real
 * arithmetic are written as one canonical double-precision expression each.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), key = (seed low, seed high):
 *   Gibbs update of spin v at sweep t in grid position p:
 *       counter (rho(v) >> 2, t, p, 0), output word rho(v) & 3
 *   swap of pair (k, k+1) on line `line` in round n, direction d (0 = P, 1 = beta):
 *       counter (k, n, line, 1 + d), u = ((x0 >> 5) 2^26 + (x1 >> 6)) 2^-53
 *   initial spin v at position p when no initial state is given:
 *       counter (v >> 2, 0, p, 3), output word v & 3, +1 iff its top bit is set
 * rho(v) is v's rank after sorting spins by (colour, index), every colour's
 * first rank being rounded up to a multiple of 4.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2

#define ORACLE_NO_PSWAP 1u

/* Threads that share the replicas' sweeps inside a round (1 by default).
 * Positions are independent during the sweep phase and every random number
 * is keyed by position, so the result does not depend on this; the swap
 * step and tracking stay sequential.  Without OpenMP the pragma is ignored
 * and the run is single-threaded. */
static int32_t oracle_threads = 1;

void oracle_set_threads(int32_t threads) { oracle_threads = threads > 0 ? threads : 1; }

/* ---------------------------------------------------------------- Philox */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t philox_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                            uint32_t c3, int which)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[which];
}

static double philox_u53(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    double hi = (double)(out[0] >> 5);
    double lo = (double)(out[1] >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------------- colour ranks */

/* rank[v] for every spin; returns the padded total through n_pad. */
int oracle_color_rank(int32_t n, const int32_t *color, int32_t *rank, int32_t *n_pad)
{
    int32_t n_colors = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (color[v] < 0) return ORACLE_EINVAL;
        if (color[v] + 1 > n_colors) n_colors = color[v] + 1;
    }
    int64_t base = 0;
    for (int32_t c = 0; c < n_colors; ++c) {
        int64_t next = base;
        for (int32_t v = 0; v < n; ++v) {
            if (color[v] == c) rank[v] = (int32_t)next++;
        }
        int64_t size = next - base;
        base += (size + 3) / 4 * 4;
    }
    *n_pad = (int32_t)base;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- energy */

typedef struct {
    int32_t n;
    const int32_t *row_ptr, *col, *J_q, *b_q;
    int32_t m;
    const int32_t *copy_a, *copy_b;
    const int32_t *color;
} oracle_instance;

/* f = -sum_{i<j} J_ij s_i s_j - sum_i b_i s_i ; g = sum_copy (s_a - s_b)^2 */
void oracle_energy(int32_t n, const int32_t *row_ptr, const int32_t *col,
                   const int32_t *J_q, const int32_t *b_q, int32_t m,
                   const int32_t *copy_a, const int32_t *copy_b,
                   const int8_t *s, int64_t *f_out, int64_t *g_out)
{
    int64_t f = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            if (j > i) f -= (int64_t)J_q[e] * s[i] * s[j];
        }
        if (b_q) f -= (int64_t)b_q[i] * s[i];
    }
    int64_t g = 0;
    for (int32_t e = 0; e < m; ++e) {
        int64_t d = (int64_t)s[copy_a[e]] - s[copy_b[e]];
        g += d * d;
    }
    *f_out = f;
    *g_out = g;
}

/* General constraints: g = sum_t r_t^2 with r_t = sum_{k} a_tk s_{i_tk} + d_t,
 * term t holding entries term_ptr[t] .. term_ptr[t+1]-1 of term_idx /
 * term_coef. */
static int64_t term_residual(const int32_t *term_ptr, const int32_t *term_idx,
                             const int32_t *term_coef, const int32_t *term_const,
                             int32_t t, const int8_t *s)
{
    int64_t r = term_const[t];
    for (int32_t e = term_ptr[t]; e < term_ptr[t + 1]; ++e)
        r += (int64_t)term_coef[e] * s[term_idx[e]];
    return r;
}

/* f as in oracle_energy, g = sum_t r_t^2 */
void oracle_energy_terms(int32_t n, const int32_t *row_ptr, const int32_t *col,
                         const int32_t *J_q, const int32_t *b_q, int32_t n_terms,
                         const int32_t *term_ptr, const int32_t *term_idx,
                         const int32_t *term_coef, const int32_t *term_const,
                         const int8_t *s, int64_t *f_out, int64_t *g_out)
{
    int64_t f, g_unused;
    oracle_energy(n, row_ptr, col, J_q, b_q, 0, NULL, NULL, s, &f, &g_unused);
    int64_t g = 0;
    for (int32_t t = 0; t < n_terms; ++t) {
        int64_t r = term_residual(term_ptr, term_idx, term_coef, term_const, t, s);
        g += r * r;
    }
    *f_out = f;
    *g_out = g;
}

/* The constraint of a run: copy edges (n_terms < 0) or general terms, with
 * the list of (term, entry) incidences of every spin for the latter. */
typedef struct {
    int32_t m;
    const int32_t *copy_a, *copy_b;
    int32_t *chain_ptr, *chain_nbr;   /* copy neighbours of every spin */
    int32_t n_terms;                  /* -1: copy edges */
    const int32_t *term_ptr, *term_idx, *term_coef, *term_const;
    int32_t *inc_ptr, *inc_entry;     /* entries of term_idx naming each spin */
    int32_t *entry_term;              /* term of every entry */
} oracle_constraint;

static int constraint_init(oracle_constraint *c, int32_t n)
{
    c->chain_ptr = c->chain_nbr = c->inc_ptr = c->inc_entry = c->entry_term = NULL;
    if (c->n_terms < 0) {
        c->chain_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        c->chain_nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * c->m + 1));
        int32_t *fill = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        if (!c->chain_ptr || !c->chain_nbr || !fill) { free(fill); return ORACLE_ENOMEM; }
        for (int32_t e = 0; e < c->m; ++e) {
            c->chain_ptr[c->copy_a[e] + 1]++;
            c->chain_ptr[c->copy_b[e] + 1]++;
        }
        for (int32_t v = 0; v < n; ++v) c->chain_ptr[v + 1] += c->chain_ptr[v];
        for (int32_t e = 0; e < c->m; ++e) {
            int32_t a = c->copy_a[e], b = c->copy_b[e];
            c->chain_nbr[c->chain_ptr[a] + fill[a]++] = b;
            c->chain_nbr[c->chain_ptr[b] + fill[b]++] = a;
        }
        free(fill);
        return ORACLE_OK;
    }
    const int32_t ne = c->term_ptr[c->n_terms];
    c->inc_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    c->inc_entry = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
    c->entry_term = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
    int32_t *fill = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!c->inc_ptr || !c->inc_entry || !c->entry_term || !fill) { free(fill); return ORACLE_ENOMEM; }
    for (int32_t t = 0; t < c->n_terms; ++t)
        for (int32_t e = c->term_ptr[t]; e < c->term_ptr[t + 1]; ++e) {
            c->entry_term[e] = t;
            c->inc_ptr[c->term_idx[e] + 1]++;
        }
    for (int32_t v = 0; v < n; ++v) c->inc_ptr[v + 1] += c->inc_ptr[v];
    for (int32_t e = 0; e < ne; ++e) {
        int32_t v = c->term_idx[e];
        c->inc_entry[c->inc_ptr[v] + fill[v]++] = e;
    }
    free(fill);
    return ORACLE_OK;
}

static void constraint_free(oracle_constraint *c)
{
    free(c->chain_ptr); free(c->chain_nbr);
    free(c->inc_ptr); free(c->inc_entry); free(c->entry_term);
}

/* c_v: the factor of P in spin v's local field (E = -s_v (h_v) + terms free
 * of s_v).  Copy edges: 2 sum of the copies.  Terms: the part of
 * (a s_v + rest)^2 that depends on s_v is 2 a s_v rest, so
 * c_v = -2 sum_t a_tv rest_t with rest_t = r_t - a_tv s_v. */
static int64_t constraint_field(const oracle_constraint *c, const int8_t *s, int32_t v)
{
    if (c->n_terms < 0) {
        int64_t cs = 0;
        for (int32_t e = c->chain_ptr[v]; e < c->chain_ptr[v + 1]; ++e) cs += s[c->chain_nbr[e]];
        return 2 * cs;
    }
    int64_t acc = 0;
    for (int32_t k = c->inc_ptr[v]; k < c->inc_ptr[v + 1]; ++k) {
        const int32_t e = c->inc_entry[k], t = c->entry_term[e];
        const int64_t a = c->term_coef[e];
        const int64_t rest = term_residual(c->term_ptr, c->term_idx, c->term_coef, c->term_const, t, s)
                             - a * s[v];
        acc += a * rest;
    }
    return -2 * acc;
}

static void constraint_energy(const oracle_constraint *c, int32_t n, const int32_t *row_ptr,
                              const int32_t *col, const int32_t *J_q, const int32_t *b_q,
                              const int8_t *s, int64_t *f, int64_t *g)
{
    if (c->n_terms < 0)
        oracle_energy(n, row_ptr, col, J_q, b_q, c->m, c->copy_a, c->copy_b, s, f, g);
    else
        oracle_energy_terms(n, row_ptr, col, J_q, b_q, c->n_terms, c->term_ptr, c->term_idx,
                            c->term_coef, c->term_const, s, f, g);
}

/* ------------------------------------------------------------ swap rules */

/* Eq. 2: exponent of a P-swap between penalty columns a (left) and b (right)
 * of the same row: beta (P_b - P_a) (g_b - g_a), penalties in Q12. */
double oracle_pswap_exponent(double beta, int32_t pq_a, int32_t pq_b, int64_t g_a, int64_t g_b)
{
    int64_t dpg = ((int64_t)pq_b - pq_a) * (g_b - g_a);
    return ldexp(beta * (double)dpg, -12);
}

/* Eq. 3: exponent of a beta-swap between rows a (upper) and b (lower) of the
 * same column: (beta_b - beta_a) (E_b - E_a), energies in Q12. */
double oracle_bswap_exponent(double beta_a, double beta_b, int64_t e_a, int64_t e_b)
{
    double dbeta = beta_b - beta_a;
    return ldexp(dbeta * (double)(e_b - e_a), -12);
}

/* Metropolis test "rand <= min(1, exp(x))" with rand in [0, 1). */
int oracle_swap_accept(double x, double u)
{
    if (x >= 0.0) return 1;
    return u <= exp(x);
}

/* Heat-bath decision for a spin with Q12 local field h at inverse
 * temperature beta, given a 32-bit uniform: +1 with probability
 * sigma(2 beta h) = 1 / (1 + exp(-2 beta h)). */
int oracle_heat_bath(double beta, int64_t h_q, uint32_t u)
{
    double x = ldexp(beta * (double)h_q, -11);
    double p = 1.0 / (1.0 + exp(-x));
    return ((double)u < ldexp(p, 32)) ? 1 : -1;
}

/* Swap direction and pair parity of round n (1-based) under Algorithm 1:
 * the direction starts on P and flips after every even round; the first
 * left index is 1 on even rounds, 0 on odd ones (0-based). */
void oracle_schedule(int64_t n, uint32_t flags, int32_t *dir_beta, int32_t *first)
{
    int even = (n % 2 == 0);
    *first = even ? 1 : 0;
    if (flags & ORACLE_NO_PSWAP) {
        *dir_beta = 1;
    } else {
        *dir_beta = (((n - 1) / 2) % 2 == 1);
    }
}

/* -------------------------------------------------------------- the run */

typedef struct {
    int8_t *states;      /* [R * n], position order, written at the end */
    int64_t *f, *g;      /* [R], position order */
    int8_t *best_state;  /* [n] */
    int64_t best_f, best_sweep, first_hit;
    int64_t *p_att, *p_acc; /* [I * (J-1)], row-major (row, left index) */
    int64_t *b_att, *b_acc; /* [J * (I-1)], (column, left index) */
    int64_t *trace_f, *trace_g; /* [trace_cap] bottom-right f, g per round */
    int64_t trace_cap;
} oracle_out;

static int run_core(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *J_q,
               const int32_t *b_q, oracle_constraint *cons,
               const int32_t *color,
               int32_t n_beta, const double *beta, int32_t n_p, const int32_t *p_q,
               int32_t mcs_per_swap, int64_t n_rounds, uint64_t seed,
               const int8_t *s0, int32_t has_target, int64_t f_target, uint32_t flags,
               int8_t *states_out, int64_t *f_out, int64_t *g_out,
               int8_t *best_state, int64_t *best_f, int64_t *best_sweep, int64_t *first_hit,
               int64_t *p_att, int64_t *p_acc, int64_t *b_att, int64_t *b_acc,
               int64_t *trace_f, int64_t *trace_g, int64_t trace_cap)
{
    if (n <= 0 || n_beta <= 0 || n_p <= 0 || mcs_per_swap <= 0 || n_rounds < 0)
        return ORACLE_EINVAL;
    const int32_t R = n_beta * n_p;
    int32_t n_colors = 0;
    for (int32_t v = 0; v < n; ++v)
        if (color[v] + 1 > n_colors) n_colors = color[v] + 1;

    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *class_start = (int32_t *)calloc((size_t)n_colors + 1, sizeof(int32_t));
    int8_t *pool = (int8_t *)malloc((size_t)R * (size_t)n);
    int8_t **state = (int8_t **)malloc(sizeof(int8_t *) * (size_t)R);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    if (!rank || !order || !class_start || !pool || !state || !f || !g ||
        constraint_init(cons, n) != ORACLE_OK) {
        free(rank); free(order); free(class_start);
        free(pool); free(state); free(f); free(g);
        constraint_free(cons);
        return ORACLE_ENOMEM;
    }
    int32_t n_pad;
    oracle_color_rank(n, color, rank, &n_pad);
    (void)n_pad;

    /* spins of each colour class in ascending index */
    {
        int32_t k = 0;
        for (int32_t c = 0; c < n_colors; ++c) {
            class_start[c] = k;
            for (int32_t v = 0; v < n; ++v)
                if (color[v] == c) order[k++] = v;
        }
        class_start[n_colors] = k;
    }
    /* initial configurations, one per grid position */
    for (int32_t p = 0; p < R; ++p) {
        state[p] = pool + (size_t)p * (size_t)n;
        for (int32_t v = 0; v < n; ++v) {
            if (s0) {
                state[p][v] = s0[(size_t)p * (size_t)n + (size_t)v];
            } else {
                uint32_t w = philox_word(seed, (uint32_t)v >> 2, 0u, (uint32_t)p, 3u, v & 3);
                state[p][v] = (w >> 31) ? 1 : -1;
            }
        }
    }

    if (p_att) memset(p_att, 0, sizeof(int64_t) * (size_t)(n_beta * (n_p - 1 > 0 ? n_p - 1 : 0)));
    if (p_acc) memset(p_acc, 0, sizeof(int64_t) * (size_t)(n_beta * (n_p - 1 > 0 ? n_p - 1 : 0)));
    if (b_att) memset(b_att, 0, sizeof(int64_t) * (size_t)(n_p * (n_beta - 1 > 0 ? n_beta - 1 : 0)));
    if (b_acc) memset(b_acc, 0, sizeof(int64_t) * (size_t)(n_p * (n_beta - 1 > 0 ? n_beta - 1 : 0)));
    int64_t bf = INT64_MAX, bsweep = -1, fhit = -1;
    const int32_t br = R - 1;

    for (int32_t p = 0; p < R; ++p)
        constraint_energy(cons, n, row_ptr, col, J_q, b_q, state[p], &f[p], &g[p]);

    for (int64_t rnd = 1; rnd <= n_rounds; ++rnd) {
        /* every replica performs mcs_per_swap sweeps */
#pragma omp parallel for num_threads(oracle_threads) schedule(dynamic, 1)
        for (int32_t p = 0; p < R; ++p) {
            const int32_t i = p / n_p, j = p % n_p;
            int8_t *s = state[p];
            for (int32_t k = 0; k < mcs_per_swap; ++k) {
                const uint32_t t = (uint32_t)((rnd - 1) * mcs_per_swap + k);
                for (int32_t c = 0; c < n_colors; ++c) {
                    for (int32_t q = class_start[c]; q < class_start[c + 1]; ++q) {
                        const int32_t v = order[q];
                        int64_t h = b_q ? b_q[v] : 0;
                        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
                            h += (int64_t)J_q[e] * s[col[e]];
                        h += (int64_t)p_q[j] * constraint_field(cons, s, v);
                        uint32_t u = philox_word(seed, (uint32_t)rank[v] >> 2, t, (uint32_t)p,
                                                 0u, rank[v] & 3);
                        s[v] = (int8_t)oracle_heat_bath(beta[i], h, u);
                    }
                }
            }
            /* "for final sweep: compute energy E and constraint g" */
            constraint_energy(cons, n, row_ptr, col, J_q, b_q, s, &f[p], &g[p]);
        }

        int32_t dir_beta, first;
        oracle_schedule(rnd, flags, &dir_beta, &first);
        if (!dir_beta) {
            for (int32_t i = 0; i < n_beta; ++i) {
                for (int32_t k = first; k + 1 < n_p; k += 2) {
                    const int32_t a = i * n_p + k, b = a + 1;
                    double x = oracle_pswap_exponent(beta[i], p_q[k], p_q[k + 1], g[a], g[b]);
                    double u = philox_u53(seed, (uint32_t)k, (uint32_t)rnd, (uint32_t)i, 1u);
                    int acc = oracle_swap_accept(x, u);
                    if (p_att) p_att[i * (n_p - 1) + k]++;
                    if (acc) {
                        if (p_acc) p_acc[i * (n_p - 1) + k]++;
                        int8_t *ts = state[a]; state[a] = state[b]; state[b] = ts;
                        int64_t tf = f[a]; f[a] = f[b]; f[b] = tf;
                        int64_t tg = g[a]; g[a] = g[b]; g[b] = tg;
                    }
                }
            }
        } else {
            for (int32_t j = 0; j < n_p; ++j) {
                for (int32_t k = first; k + 1 < n_beta; k += 2) {
                    const int32_t a = k * n_p + j, b = a + n_p;
                    int64_t ea = f[a] + (int64_t)p_q[j] * g[a];
                    int64_t eb = f[b] + (int64_t)p_q[j] * g[b];
                    double x = oracle_bswap_exponent(beta[k], beta[k + 1], ea, eb);
                    double u = philox_u53(seed, (uint32_t)k, (uint32_t)rnd, (uint32_t)j, 2u);
                    int acc = oracle_swap_accept(x, u);
                    if (b_att) b_att[j * (n_beta - 1) + k]++;
                    if (acc) {
                        if (b_acc) b_acc[j * (n_beta - 1) + k]++;
                        int8_t *ts = state[a]; state[a] = state[b]; state[b] = ts;
                        int64_t tf = f[a]; f[a] = f[b]; f[b] = tf;
                        int64_t tg = g[a]; g[a] = g[b]; g[b] = tg;
                    }
                }
            }
        }

        /* "store spins from the last replica": the bottom-right position */
        const int64_t sweeps_done = rnd * mcs_per_swap;
        if (trace_f && rnd - 1 < trace_cap) trace_f[rnd - 1] = f[br];
        if (trace_g && rnd - 1 < trace_cap) trace_g[rnd - 1] = g[br];
        if (g[br] == 0) {
            if (has_target && fhit < 0 && f[br] <= f_target) fhit = sweeps_done;
            if (f[br] < bf) {
                bf = f[br];
                bsweep = sweeps_done;
                if (best_state) memcpy(best_state, state[br], (size_t)n);
            }
        }
    }

    if (states_out)
        for (int32_t p = 0; p < R; ++p)
            memcpy(states_out + (size_t)p * (size_t)n, state[p], (size_t)n);
    if (f_out) memcpy(f_out, f, sizeof(int64_t) * (size_t)R);
    if (g_out) memcpy(g_out, g, sizeof(int64_t) * (size_t)R);
    if (best_f) *best_f = bf;
    if (best_sweep) *best_sweep = bsweep;
    if (first_hit) *first_hit = fhit;

    free(rank); free(order); free(class_start);
    free(pool); free(state); free(f); free(g);
    constraint_free(cons);
    return ORACLE_OK;
}

#define RUN_TAIL_PARAMS                                                                         \
    const int32_t *color, int32_t n_beta, const double *beta, int32_t n_p, const int32_t *p_q,  \
        int32_t mcs_per_swap, int64_t n_rounds, uint64_t seed, const int8_t *s0,                \
        int32_t has_target, int64_t f_target, uint32_t flags, int8_t *states_out,               \
        int64_t *f_out, int64_t *g_out, int8_t *best_state, int64_t *best_f,                    \
        int64_t *best_sweep, int64_t *first_hit, int64_t *p_att, int64_t *p_acc,                \
        int64_t *b_att, int64_t *b_acc, int64_t *trace_f, int64_t *trace_g, int64_t trace_cap
#define RUN_TAIL_ARGS                                                                           \
    color, n_beta, beta, n_p, p_q, mcs_per_swap, n_rounds, seed, s0, has_target, f_target,      \
        flags, states_out, f_out, g_out, best_state, best_f, best_sweep, first_hit, p_att,      \
        p_acc, b_att, b_acc, trace_f, trace_g, trace_cap

/* Copy-edge constraints: g = sum (s_a - s_b)^2. */
int oracle_run(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *J_q,
               const int32_t *b_q, int32_t m, const int32_t *copy_a, const int32_t *copy_b,
               RUN_TAIL_PARAMS)
{
    oracle_constraint c;
    memset(&c, 0, sizeof c);
    c.m = m;
    c.copy_a = copy_a;
    c.copy_b = copy_b;
    c.n_terms = -1;
    return run_core(n, row_ptr, col, J_q, b_q, &c, RUN_TAIL_ARGS);
}

/* General constraints: g = sum_t (sum a_ti s_i + d_t)^2. */
int oracle_run_terms(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *J_q,
                     const int32_t *b_q, int32_t n_terms, const int32_t *term_ptr,
                     const int32_t *term_idx, const int32_t *term_coef,
                     const int32_t *term_const, RUN_TAIL_PARAMS)
{
    if (n_terms < 0 || n <= 0) return ORACLE_EINVAL;
    /* every spin at most once per term */
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!seen) return ORACLE_ENOMEM;
    for (int32_t v = 0; v < n; ++v) seen[v] = -1;
    for (int32_t t = 0; t < n_terms; ++t)
        for (int32_t e = term_ptr[t]; e < term_ptr[t + 1]; ++e) {
            const int32_t v = term_idx[e];
            if (v < 0 || v >= n || seen[v] == t) { free(seen); return ORACLE_EINVAL; }
            seen[v] = t;
        }
    free(seen);
    oracle_constraint c;
    memset(&c, 0, sizeof c);
    c.n_terms = n_terms;
    c.term_ptr = term_ptr;
    c.term_idx = term_idx;
    c.term_coef = term_coef;
    c.term_const = term_const;
    return run_core(n, row_ptr, col, J_q, b_q, &c, RUN_TAIL_ARGS);
}
