/*
 * sg_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU model of colour-ordered single-spin-flip
 * descent on hyper-Ising instances with 2-spin couplings J, fields h and
 * 3-spin hyper-couplings K.  It exists to check the HIP library; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the library.
 *
 * What it follows (García & Markov, "High-performance Energy Minimization in
 * Spin-glasses with Applications to Adiabatic Quantum Computing"):
 *   - energy: Sec. II eq. (1), extended by Sec. VI eq. (5) to couplings over
 *     three spins; every undirected edge and every triple counted once;
 *   - move gain: Sec. IV, a single-spin move whose energy change is negative
 *     has positive gain; here dE_i = E(s with s_i negated) - E(s) = 2 s_i f_i
 *     with f_i = h_i + sum_j J_ij s_j + sum_(j,k) K_ijk s_j s_k;
 *   - random start drawn uniformly (Sec. IV), stop when a pass brings no
 *     improvement (Sec. IV, Fig. 3), independent starts with the best kept
 *     (Sec. IV, Sec. V);
 *   - the unfrustrated ground-state energy -sum|J| (Sec. II) and the lower
 *     bound eq. (2) are used by the tests that pin this file.
 * The paper's own pass is sequential with a gain heap; the schedule here is
 * the colour-ordered sweep (Gauss-Seidel over colour classes), with the
 * readings listed in the design notes:
 *   colouring  given, else first-fit over increasing spin index on the
 *              primal graph (edges plus the three pairs of every triple);
 *   order      colours ascending, spins of one colour ascending;
 *   rule       GREEDY flips iff dE < 0; GREEDY_TIE also flips when dE == 0
 *              and bit 0 of word 0 of Philox4x32-10(seed; i, sweep, id, r)
 *              is 1;
 *   start      s_i = -1 iff bit 0 of word 0 of
 *              Philox4x32-10(seed; i, 0xFFFFFFFF, id, r) is 1;
 *   stop       until_converged: after the first sweep with zero flips (that
 *              sweep counts); otherwise exactly max_sweeps sweeps.  A replica
 *              that converged stays frozen until it is restarted.
 * It also models the paper's own pass (oracle_fm below): max-gain moves with
 * locking and hill-climbing, best prefix kept, passes until no improvement.
 */
#include <stdint.h>
#include <limits.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11).  Counter-based: 4x32-bit counter,
 * 2x32-bit key, ten rounds; each round multiplies counter words 0 and 2 by
 * fixed odd constants, mixes the high halves with words 1 and 3 and the key,
 * and the key is advanced by two Weyl constants between rounds. */

static void oracle_mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint32_t hi0, lo0, hi1, lo1;
        oracle_mulhilo(M0, c0, &hi0, &lo0);
        oracle_mulhilo(M1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static int oracle_bit(uint64_t seed, uint32_t spin, uint32_t word1, uint32_t id, uint32_t r)
{
    uint32_t ctr[4] = {spin, word1, id, r};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return (int)(out[0] & 1u);
}

/* Fill out[4*count] with Philox outputs for counters (c0+i, c1, c2, c3). */
void oracle_philox_stream(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                          int64_t count, uint32_t* out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < count; ++i) {
        uint32_t ctr[4] = {c0 + (uint32_t)i, c1, c2, c3};
        oracle_philox4x32_10(ctr, key, out + 4 * i);
    }
}

/* ---------------------------------------------------------------------- */
/* Energy, Sec. II eq. (1) with the 3-spin terms of Sec. VI eq. (5):
 *   E(s) = - sum_edges J s_i s_j - sum_i h_i s_i - sum_triples K s_i s_j s_k
 * straight from the input lists, each term once. */
int64_t oracle_energy(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej,
                      const int32_t* J, const int32_t* h, int64_t t,
                      const int32_t* tri, const int32_t* K, const int8_t* s)
{
    int64_t e = 0;
    for (int64_t k = 0; k < m; ++k)
        e -= (int64_t)J[k] * s[ei[k]] * s[ej[k]];
    if (h)
        for (int32_t i = 0; i < n; ++i)
            e -= (int64_t)h[i] * s[i];
    for (int64_t k = 0; k < t; ++k)
        e -= (int64_t)K[k] * s[tri[3 * k]] * s[tri[3 * k + 1]] * s[tri[3 * k + 2]];
    return e;
}

/* ---------------------------------------------------------------------- */
/* Incidence lists: for each spin, its couplings (partner, J) and the
 * triples it belongs to (other two members, K).  Plain arrays of lists. */
typedef struct {
    int32_t n;
    int64_t* estart;  /* n+1 */
    int32_t* epart;
    int32_t* eJ;
    int64_t* tstart;  /* n+1 */
    int32_t* ta;
    int32_t* tb;
    int32_t* tK;
    int32_t nc;       /* number of colours */
    int64_t* cstart;  /* nc+1 */
    int32_t* cmember; /* spins grouped by colour, ascending inside a colour */
} oracle_graph;

static void oracle_graph_free(oracle_graph* g)
{
    free(g->estart); free(g->epart); free(g->eJ);
    free(g->tstart); free(g->ta); free(g->tb); free(g->tK);
    free(g->cstart); free(g->cmember);
}

static int oracle_graph_build(oracle_graph* g, int32_t n, int64_t m, const int32_t* ei,
                              const int32_t* ej, const int32_t* J, int64_t t,
                              const int32_t* tri, const int32_t* K)
{
    memset(g, 0, sizeof(*g));
    g->n = n;
    g->estart = calloc((size_t)n + 1, sizeof(int64_t));
    g->tstart = calloc((size_t)n + 1, sizeof(int64_t));
    g->epart = malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->eJ = malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->ta = malloc(sizeof(int32_t) * (size_t)(3 * t + 1));
    g->tb = malloc(sizeof(int32_t) * (size_t)(3 * t + 1));
    g->tK = malloc(sizeof(int32_t) * (size_t)(3 * t + 1));
    if (!g->estart || !g->tstart || !g->epart || !g->eJ || !g->ta || !g->tb || !g->tK)
        return -1;
    for (int64_t k = 0; k < m; ++k) {
        g->estart[ei[k] + 1]++;
        g->estart[ej[k] + 1]++;
    }
    for (int64_t k = 0; k < t; ++k)
        for (int q = 0; q < 3; ++q)
            g->tstart[tri[3 * k + q] + 1]++;
    for (int32_t i = 0; i < n; ++i) {
        g->estart[i + 1] += g->estart[i];
        g->tstart[i + 1] += g->tstart[i];
    }
    int64_t* fe = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t* ft = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fe || !ft) { free(fe); free(ft); return -1; }
    memcpy(fe, g->estart, sizeof(int64_t) * ((size_t)n + 1));
    memcpy(ft, g->tstart, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t k = 0; k < m; ++k) {
        int32_t a = ei[k], b = ej[k];
        g->epart[fe[a]] = b; g->eJ[fe[a]++] = J[k];
        g->epart[fe[b]] = a; g->eJ[fe[b]++] = J[k];
    }
    for (int64_t k = 0; k < t; ++k) {
        int32_t a = tri[3 * k], b = tri[3 * k + 1], c = tri[3 * k + 2];
        g->ta[ft[a]] = b; g->tb[ft[a]] = c; g->tK[ft[a]++] = K[k];
        g->ta[ft[b]] = a; g->tb[ft[b]] = c; g->tK[ft[b]++] = K[k];
        g->ta[ft[c]] = a; g->tb[ft[c]] = b; g->tK[ft[c]++] = K[k];
    }
    free(fe); free(ft);
    return 0;
}

/* First-fit colouring over increasing spin index on the primal graph:
 * colour[i] = smallest c >= 0 not used by any primal neighbour j < i.
 * Returns the number of colours, or -1 on allocation failure. */
static int32_t oracle_first_fit_graph(const oracle_graph* g, int32_t* colour)
{
    int32_t n = g->n, nc = 0;
    int32_t cap = 64;
    int32_t* mark = calloc((size_t)cap, sizeof(int32_t)); /* mark[c] == i+1 -> used */
    if (!mark) return -1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t stamp = i + 1;
        for (int pass = 0; pass < 2; ++pass) {
            /* pass 0: edge partners, pass 1: triple partners */
            int64_t lo = pass ? g->tstart[i] : g->estart[i];
            int64_t hi = pass ? g->tstart[i + 1] : g->estart[i + 1];
            for (int64_t q = lo; q < hi; ++q) {
                int32_t others[2];
                int cnt;
                if (pass == 0) { others[0] = g->epart[q]; cnt = 1; }
                else { others[0] = g->ta[q]; others[1] = g->tb[q]; cnt = 2; }
                for (int u = 0; u < cnt; ++u) {
                    int32_t j = others[u];
                    if (j < i) {
                        int32_t c = colour[j];
                        if (c >= cap) {
                            int32_t ncap = cap;
                            while (ncap <= c) ncap *= 2;
                            int32_t* nm = realloc(mark, sizeof(int32_t) * (size_t)ncap);
                            if (!nm) { free(mark); return -1; }
                            memset(nm + cap, 0, sizeof(int32_t) * (size_t)(ncap - cap));
                            mark = nm; cap = ncap;
                        }
                        mark[c] = stamp;
                    }
                }
            }
        }
        int32_t c = 0;
        while (c < cap && mark[c] == stamp) ++c;
        colour[i] = c;
        if (c + 1 > nc) nc = c + 1;
        if (nc >= cap) {
            int32_t* nm = realloc(mark, sizeof(int32_t) * (size_t)cap * 2);
            if (!nm) { free(mark); return -1; }
            memset(nm + cap, 0, sizeof(int32_t) * (size_t)cap);
            mark = nm; cap *= 2;
        }
    }
    free(mark);
    return nc;
}

/* 1 if no two primal neighbours share a colour, else 0. */
static int oracle_proper_graph(const oracle_graph* g, const int32_t* colour)
{
    for (int32_t i = 0; i < g->n; ++i) {
        if (colour[i] < 0) return 0;
        for (int64_t q = g->estart[i]; q < g->estart[i + 1]; ++q)
            if (colour[g->epart[q]] == colour[i]) return 0;
        for (int64_t q = g->tstart[i]; q < g->tstart[i + 1]; ++q)
            if (colour[g->ta[q]] == colour[i] || colour[g->tb[q]] == colour[i]) return 0;
    }
    return 1;
}

int32_t oracle_first_fit_colouring(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej,
                                   int64_t t, const int32_t* tri, int32_t* colour_out)
{
    oracle_graph g;
    int32_t* zeroJ = calloc((size_t)m + 1, sizeof(int32_t));
    int32_t* zeroK = calloc((size_t)t + 1, sizeof(int32_t));
    int32_t nc = -1;
    if (zeroJ && zeroK && oracle_graph_build(&g, n, m, ei, ej, zeroJ, t, tri, zeroK) == 0)
        nc = oracle_first_fit_graph(&g, colour_out);
    oracle_graph_free(&g);
    free(zeroJ); free(zeroK);
    return nc;
}

int oracle_colouring_is_proper(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej,
                               int64_t t, const int32_t* tri, const int32_t* colour)
{
    oracle_graph g;
    int32_t* zeroJ = calloc((size_t)m + 1, sizeof(int32_t));
    int32_t* zeroK = calloc((size_t)t + 1, sizeof(int32_t));
    int ok = -1;
    if (zeroJ && zeroK && oracle_graph_build(&g, n, m, ei, ej, zeroJ, t, tri, zeroK) == 0)
        ok = oracle_proper_graph(&g, colour);
    oracle_graph_free(&g);
    free(zeroJ); free(zeroK);
    return ok;
}

static int oracle_group_colours(oracle_graph* g, const int32_t* colour)
{
    int32_t nc = 0;
    for (int32_t i = 0; i < g->n; ++i)
        if (colour[i] + 1 > nc) nc = colour[i] + 1;
    g->nc = nc;
    g->cstart = calloc((size_t)nc + 1, sizeof(int64_t));
    g->cmember = malloc(sizeof(int32_t) * ((size_t)g->n + 1));
    if (!g->cstart || !g->cmember) return -1;
    for (int32_t i = 0; i < g->n; ++i) g->cstart[colour[i] + 1]++;
    for (int32_t c = 0; c < nc; ++c) g->cstart[c + 1] += g->cstart[c];
    int64_t* fill = malloc(sizeof(int64_t) * ((size_t)nc + 1));
    if (!fill) return -1;
    memcpy(fill, g->cstart, sizeof(int64_t) * ((size_t)nc + 1));
    for (int32_t i = 0; i < g->n; ++i) g->cmember[fill[colour[i]]++] = i;
    free(fill);
    return 0;
}

/* Local field of spin i: f_i = h_i + sum_j J_ij s_j + sum K s_j s_k. */
static int64_t oracle_field(const oracle_graph* g, const int32_t* h, const int8_t* s, int32_t i)
{
    int64_t f = h ? h[i] : 0;
    for (int64_t q = g->estart[i]; q < g->estart[i + 1]; ++q)
        f += (int64_t)g->eJ[q] * s[g->epart[q]];
    for (int64_t q = g->tstart[i]; q < g->tstart[i + 1]; ++q)
        f += (int64_t)g->tK[q] * s[g->ta[q]] * s[g->tb[q]];
    return f;
}

/* Sweep orders inside a colour class (all must give identical results under
 * a proper colouring; the tests use this to check that claim). */
enum { ORDER_ASCENDING = 0, ORDER_DESCENDING = 1, ORDER_SIMULTANEOUS = 2 };

typedef struct {
    uint64_t seed;
    int32_t rule;           /* 0 GREEDY, 1 GREEDY_TIE */
    int32_t max_sweeps;     /* sweeps allowed in this call */
    int32_t until_converged;
    int32_t order;
    uint32_t instance_id;
} oracle_params;

/* One replica.  Returns 1 if it converged in this call or was already
 * converged, 0 otherwise.  *E is the tracked energy (in/out), *sweeps and
 * *flips are cumulative counters, trace_E (optional) receives the tracked
 * energy after every colour phase, trace_s (optional) the spins. */
static int oracle_replica(const oracle_graph* g, const int32_t* h, const oracle_params* p,
                          uint32_t restart, int8_t* s, int64_t* E, int64_t* sweeps,
                          int64_t* flips, int8_t* converged, int64_t* trace_E,
                          int8_t* trace_s, int64_t trace_cap, int64_t* trace_len,
                          int8_t* scratch)
{
    if (*converged) return 1;
    int64_t tl = 0;
    for (int32_t done = 0; done < p->max_sweeps; ++done) {
        uint32_t sweep = (uint32_t)(*sweeps);
        int64_t F = 0;
        for (int32_t c = 0; c < g->nc; ++c) {
            int64_t lo = g->cstart[c], hi = g->cstart[c + 1];
            if (p->order == ORDER_SIMULTANEOUS) {
                /* decide every spin of the colour from the state before the
                 * phase, then apply all the flips */
                for (int64_t q = lo; q < hi; ++q) {
                    int32_t i = g->cmember[q];
                    int64_t d = 2 * (int64_t)s[i] * oracle_field(g, h, s, i);
                    int fl = d < 0 || (p->rule == 1 && d == 0 &&
                                       oracle_bit(p->seed, (uint32_t)i, sweep, p->instance_id, restart));
                    scratch[i] = (int8_t)fl;
                    if (fl) { *E += d; ++F; }
                }
                for (int64_t q = lo; q < hi; ++q) {
                    int32_t i = g->cmember[q];
                    if (scratch[i]) s[i] = (int8_t)-s[i];
                }
            } else {
                for (int64_t qq = lo; qq < hi; ++qq) {
                    int64_t q = (p->order == ORDER_DESCENDING) ? (hi - 1 - (qq - lo)) : qq;
                    int32_t i = g->cmember[q];
                    int64_t d = 2 * (int64_t)s[i] * oracle_field(g, h, s, i);
                    if (d < 0 || (p->rule == 1 && d == 0 &&
                                  oracle_bit(p->seed, (uint32_t)i, sweep, p->instance_id, restart))) {
                        s[i] = (int8_t)-s[i];
                        *E += d;
                        ++F;
                    }
                }
            }
            if (trace_E && tl < trace_cap) {
                trace_E[tl] = *E;
                if (trace_s) memcpy(trace_s + tl * g->n, s, (size_t)g->n);
                ++tl;
            }
        }
        *sweeps += 1;
        *flips += F;
        if (p->until_converged && F == 0) {
            *converged = 1;
            break;
        }
    }
    if (trace_len) *trace_len = tl;
    return *converged ? 1 : 0;
}

/*
 * Run the colour-ordered descent on every restart of one instance.
 *   colour        NULL: first-fit; else must be proper (else returns -2)
 *   init          1: draw the random start of every restart (and reset
 *                 sweeps, flips, converged); 0: continue from the given
 *                 spins and counters
 *   spins         restarts*n, external order, in/out
 *   energy        restarts, out (recomputed at entry, tracked through flips)
 *   sweeps, flips restarts, cumulative, in/out
 *   converged     restarts, in/out
 *   threads       > 0: OpenMP threads over restarts; 0: default
 * Returns 0; 1 if until_converged and some restart did not converge;
 * negative on bad input or allocation failure.
 */
int oracle_run(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej, const int32_t* J,
               const int32_t* h, int64_t t, const int32_t* tri, const int32_t* K,
               const int32_t* colour, uint32_t instance_id, int32_t restarts, uint64_t seed,
               int32_t rule, int32_t max_sweeps, int32_t until_converged, int32_t order,
               int32_t init, int8_t* spins, int64_t* energy, int64_t* sweeps, int64_t* flips,
               int8_t* converged, int32_t threads)
{
    if (n < 1 || restarts < 1 || max_sweeps < 0) return -1;
    oracle_graph g;
    if (oracle_graph_build(&g, n, m, ei, ej, J, t, tri, K) != 0) { oracle_graph_free(&g); return -3; }
    int32_t* col = malloc(sizeof(int32_t) * (size_t)n);
    if (!col) { oracle_graph_free(&g); return -3; }
    if (colour) {
        memcpy(col, colour, sizeof(int32_t) * (size_t)n);
        if (!oracle_proper_graph(&g, col)) { free(col); oracle_graph_free(&g); return -2; }
    } else if (oracle_first_fit_graph(&g, col) < 0) {
        free(col); oracle_graph_free(&g); return -3;
    }
    if (oracle_group_colours(&g, col) != 0) { free(col); oracle_graph_free(&g); return -3; }
    free(col);

    oracle_params p = {seed, rule, max_sweeps, until_converged, order, instance_id};
    int notconv = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : notconv)
#endif
    for (int32_t r = 0; r < restarts; ++r) {
        int8_t* s = spins + (int64_t)r * n;
        int8_t* scratch = (order == ORDER_SIMULTANEOUS) ? malloc((size_t)n) : NULL;
        if (init) {
            for (int32_t i = 0; i < n; ++i)
                s[i] = oracle_bit(seed, (uint32_t)i, 0xFFFFFFFFu, instance_id, (uint32_t)r) ? -1 : 1;
            sweeps[r] = 0;
            flips[r] = 0;
            converged[r] = 0;
        }
        int64_t E = oracle_energy(n, m, ei, ej, J, h, t, tri, K, s);
        int ok = oracle_replica(&g, h, &p, (uint32_t)r, s, &E, &sweeps[r], &flips[r],
                                &converged[r], NULL, NULL, 0, NULL, scratch);
        energy[r] = E;
        if (until_converged && !ok) notconv += 1;
        free(scratch);
    }
    oracle_graph_free(&g);
    return notconv ? 1 : 0;
}

/* One restart with a per-phase trace (small instances): trace_E[phase] is the
 * tracked energy after each colour phase, trace_s[phase*n ..] the spins.
 * Returns the number of recorded phases, or negative on error. */
int64_t oracle_trace(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej, const int32_t* J,
                     const int32_t* h, int64_t t, const int32_t* tri, const int32_t* K,
                     const int32_t* colour, uint32_t instance_id, uint32_t restart, uint64_t seed,
                     int32_t rule, int32_t max_sweeps, int32_t until_converged, int32_t order,
                     int32_t init, int8_t* s, int64_t* sweeps, int64_t* flips, int8_t* converged,
                     int64_t* trace_E, int8_t* trace_s, int64_t trace_cap)
{
    oracle_graph g;
    if (oracle_graph_build(&g, n, m, ei, ej, J, t, tri, K) != 0) { oracle_graph_free(&g); return -3; }
    int32_t* col = malloc(sizeof(int32_t) * (size_t)n);
    int8_t* scratch = malloc((size_t)n);
    if (!col || !scratch) { free(col); free(scratch); oracle_graph_free(&g); return -3; }
    if (colour) {
        memcpy(col, colour, sizeof(int32_t) * (size_t)n);
        if (!oracle_proper_graph(&g, col)) { free(col); free(scratch); oracle_graph_free(&g); return -2; }
    } else {
        oracle_first_fit_graph(&g, col);
    }
    oracle_group_colours(&g, col);
    free(col);
    if (init) {
        for (int32_t i = 0; i < n; ++i)
            s[i] = oracle_bit(seed, (uint32_t)i, 0xFFFFFFFFu, instance_id, restart) ? -1 : 1;
        *sweeps = 0; *flips = 0; *converged = 0;
    }
    oracle_params p = {seed, rule, max_sweeps, until_converged, order, instance_id};
    int64_t E = oracle_energy(n, m, ei, ej, J, h, t, tri, K, s);
    int64_t len = 0;
    oracle_replica(&g, h, &p, restart, s, &E, sweeps, flips, converged, trace_E, trace_s,
                   trace_cap, &len, scratch);
    free(scratch);
    oracle_graph_free(&g);
    return len;
}

/* Same as oracle_trace but with an arbitrary (possibly improper) colouring,
 * used only to show that the order tests can detect a bad colouring. */
int64_t oracle_trace_unchecked(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej,
                               const int32_t* J, const int32_t* h, int64_t t, const int32_t* tri,
                               const int32_t* K, const int32_t* colour, uint64_t seed,
                               int32_t rule, int32_t max_sweeps, int32_t order, int8_t* s,
                               int64_t* trace_E, int64_t trace_cap)
{
    oracle_graph g;
    if (oracle_graph_build(&g, n, m, ei, ej, J, t, tri, K) != 0) { oracle_graph_free(&g); return -3; }
    int8_t* scratch = malloc((size_t)n);
    oracle_group_colours(&g, colour);
    oracle_params p = {seed, rule, max_sweeps, 0, order, 0};
    int64_t E = oracle_energy(n, m, ei, ej, J, h, t, tri, K, s);
    int64_t sw = 0, fl = 0, len = 0;
    int8_t cv = 0;
    oracle_replica(&g, h, &p, 0, s, &E, &sw, &fl, &cv, trace_E, NULL, trace_cap, &len, scratch);
    free(scratch);
    oracle_graph_free(&g);
    return len;
}

/* Exhaustive ground state for n <= 30: walks all 2^n states in Gray-code
 * order, updating the energy by the single-flip change 2 s_i f_i (f from the
 * incidence lists), starting from the all-(+1) state whose energy is taken
 * from oracle_energy.  Ties keep the first state met.  Writes the minimising
 * state to best_s (may be NULL) and returns its energy; also returns the
 * number of ground states (equal minimum energy) in *degeneracy. */
int64_t oracle_brute_force(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej,
                           const int32_t* J, const int32_t* h, int64_t t, const int32_t* tri,
                           const int32_t* K, int8_t* best_s, int64_t* degeneracy)
{
    if (n < 1 || n > 30) return INT64_MIN;
    oracle_graph g;
    if (oracle_graph_build(&g, n, m, ei, ej, J, t, tri, K) != 0) { oracle_graph_free(&g); return INT64_MIN; }
    int8_t* s = malloc((size_t)n);
    for (int32_t i = 0; i < n; ++i) s[i] = 1;
    int64_t E = oracle_energy(n, m, ei, ej, J, h, t, tri, K, s);
    int64_t best = E, deg = 1;
    if (best_s) memcpy(best_s, s, (size_t)n);
    uint64_t total = (uint64_t)1 << n;
    for (uint64_t k = 1; k < total; ++k) {
        int32_t i = __builtin_ctzll(k);        /* Gray code: flip the lowest set bit of k */
        E += 2 * (int64_t)s[i] * oracle_field(&g, h, s, i);
        s[i] = (int8_t)-s[i];
        if (E < best) {
            best = E; deg = 1;
            if (best_s) memcpy(best_s, s, (size_t)n);
        } else if (E == best) {
            ++deg;
        }
    }
    free(s);
    oracle_graph_free(&g);
    if (degeneracy) *degeneracy = deg;
    return best;
}

/* ---------------------------------------------------------------------- */
/* The paper's pass-based local search with hill-climbing (Sec. IV, Fig. 3).
 * A pass starts from the state SP* and its energy.  n times: every unlocked
 * spin's gain -dE_i is evaluated from the definition (no incremental update),
 * the unlocked spin of largest gain is moved even when that gain is negative
 * (lowest spin index among equal gains), and locked; whenever the energy is
 * strictly below the lowest seen in this pass, the state is remembered.  At the
 * end of the pass the remembered state becomes SP*.  The search stops after
 * the first pass that leaves the energy of SP* unchanged (that pass counts).
 *   passes  cumulative pass count, in/out
 *   kept    cumulative number of moves kept (the length of each pass's best
 *           prefix), in/out
 * Readings: ties go to the lowest index; "energy decreased" is strict and is
 * measured against the lowest energy seen so far in the pass. */
static void oracle_fm_replica(const oracle_graph* g, const int32_t* h, int8_t* s, int64_t* E,
                              int32_t max_passes, int32_t until_converged, int64_t* passes,
                              int64_t* kept, int8_t* converged, int8_t* locked, int8_t* best)
{
    const int32_t n = g->n;
    if (*converged) return;
    for (int32_t done = 0; done < max_passes; ++done) {
        const int64_t E_start = *E;
        int64_t E_cur = *E, E_low = *E, best_len = 0;
        memcpy(best, s, (size_t)n);
        memset(locked, 0, (size_t)n);
        for (int32_t step = 0; step < n; ++step) {
            int32_t pick = -1;
            int64_t pick_gain = 0;
            for (int32_t i = 0; i < n; ++i) {
                if (locked[i]) continue;
                const int64_t gain = -2 * (int64_t)s[i] * oracle_field(g, h, s, i);
                if (pick < 0 || gain > pick_gain) {
                    pick = i;
                    pick_gain = gain;
                }
            }
            s[pick] = (int8_t)-s[pick];
            locked[pick] = 1;
            E_cur -= pick_gain;
            if (E_cur < E_low) {
                E_low = E_cur;
                best_len = step + 1;
                memcpy(best, s, (size_t)n);
            }
        }
        memcpy(s, best, (size_t)n);
        *E = E_low;
        *passes += 1;
        *kept += best_len;
        if (until_converged && !(E_low < E_start)) {
            *converged = 1;
            break;
        }
    }
}

/* The pass-based search on every restart of one instance.  init: draw the
 * random starts (same start rule as oracle_run) and reset the counters.
 * spins restarts*n external order in/out; energy out; passes, kept,
 * converged in/out.  Returns 0; 1 if until_converged and some restart did not
 * converge within max_passes; negative on bad input. */
int oracle_fm(int32_t n, int64_t m, const int32_t* ei, const int32_t* ej, const int32_t* J,
              const int32_t* h, int64_t t, const int32_t* tri, const int32_t* K, uint32_t instance_id,
              int32_t restarts, uint64_t seed, int32_t max_passes, int32_t until_converged, int32_t init,
              int8_t* spins, int64_t* energy, int64_t* passes, int64_t* kept, int8_t* converged,
              int32_t threads)
{
    if (n < 1 || restarts < 1 || max_passes < 0) return -1;
    oracle_graph g;
    if (oracle_graph_build(&g, n, m, ei, ej, J, t, tri, K) != 0) { oracle_graph_free(&g); return -3; }
    int notconv = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : notconv)
#endif
    for (int32_t r = 0; r < restarts; ++r) {
        int8_t* s = spins + (int64_t)r * n;
        int8_t* locked = malloc((size_t)n);
        int8_t* best = malloc((size_t)n);
        if (init) {
            for (int32_t i = 0; i < n; ++i)
                s[i] = oracle_bit(seed, (uint32_t)i, 0xFFFFFFFFu, instance_id, (uint32_t)r) ? -1 : 1;
            passes[r] = 0;
            kept[r] = 0;
            converged[r] = 0;
        }
        int64_t E = oracle_energy(n, m, ei, ej, J, h, t, tri, K, s);
        oracle_fm_replica(&g, h, s, &E, max_passes, until_converged, &passes[r], &kept[r], &converged[r],
                          locked, best);
        energy[r] = E;
        if (until_converged && !converged[r]) notconv += 1;
        free(locked);
        free(best);
    }
    oracle_graph_free(&g);
    return notconv ? 1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Dense hyper-Ising instances (Sec. VI eq. (5)): at most 64 spins, every
 * term a set of spins (bit i of mask[t] = spin i) with an int64 coefficient,
 * E(s) = -sum_t coef[t] * prod_{i in t} s_i; a one-spin term is a field.
 * Spins are int8 +-1 in external order.  The colour sweep uses first-fit over
 * increasing index on the primal graph (two spins adjacent when some term
 * holds both), colours ascending, spins of a colour ascending. */

static int64_t dense_prod(const int8_t* s, uint64_t m)
{
    int64_t p = 1;
    for (int i = 0; i < 64; ++i)
        if ((m >> i) & 1u) p *= s[i];
    return p;
}

int64_t oracle_dense_energy(int32_t n, int64_t nt, const uint64_t* mask, const int64_t* coef, const int8_t* s)
{
    (void)n;
    int64_t E = 0;
    for (int64_t t = 0; t < nt; ++t) E -= coef[t] * dense_prod(s, mask[t]);
    return E;
}

/* f_i = sum over terms holding i of coef * (product of the other members) */
static int64_t dense_field(int64_t nt, const uint64_t* mask, const int64_t* coef, const int8_t* s, int32_t i)
{
    int64_t f = 0;
    for (int64_t t = 0; t < nt; ++t)
        if ((mask[t] >> i) & 1u) f += coef[t] * dense_prod(s, mask[t] & ~((uint64_t)1 << i));
    return f;
}

/* spins in sweep order; returns the number of colours */
static int32_t dense_order(int32_t n, int64_t nt, const uint64_t* mask, int32_t* order)
{
    uint64_t adj[64];
    int32_t col[64];
    for (int i = 0; i < n; ++i) adj[i] = 0;
    for (int64_t t = 0; t < nt; ++t)
        for (int i = 0; i < n; ++i)
            if ((mask[t] >> i) & 1u) adj[i] |= mask[t] & ~((uint64_t)1 << i);
    int32_t nc = 0;
    for (int i = 0; i < n; ++i) {
        int c = 0;
        for (;; ++c) {
            int used = 0;
            for (int j = 0; j < i; ++j)
                if (((adj[i] >> j) & 1u) && col[j] == c) used = 1;
            if (!used) break;
        }
        col[i] = c;
        if (c + 1 > nc) nc = c + 1;
    }
    int32_t k = 0;
    for (int c = 0; c < nc; ++c)
        for (int i = 0; i < n; ++i)
            if (col[i] == c) order[k++] = i;
    return nc;
}

/* Colour sweeps (rules as oracle_run) on every restart of one dense instance.
 * init: draw the starts (bit 1 of Philox(seed; i, ~0, id, r) -> -1) and reset
 * sweeps, flips, converged.  Returns 0, 1 if until_converged and some
 * restart hit max_sweeps, negative on bad input. */
int oracle_dense_run(int32_t n, int64_t nt, const uint64_t* mask, const int64_t* coef, uint32_t instance_id,
                     int32_t restarts, uint64_t seed, int32_t rule, int32_t max_sweeps, int32_t until_converged,
                     int32_t init, int8_t* spins, int64_t* energy, int64_t* sweeps, int64_t* flips,
                     int8_t* converged)
{
    if (n < 1 || n > 64 || restarts < 1 || max_sweeps < 0) return -1;
    int32_t order[64];
    dense_order(n, nt, mask, order);
    int notconv = 0;
    for (int32_t r = 0; r < restarts; ++r) {
        int8_t* s = spins + (int64_t)r * n;
        if (init) {
            for (int32_t i = 0; i < n; ++i)
                s[i] = oracle_bit(seed, (uint32_t)i, 0xFFFFFFFFu, instance_id, (uint32_t)r) ? -1 : 1;
            sweeps[r] = 0;
            flips[r] = 0;
            converged[r] = 0;
        }
        int64_t E = oracle_dense_energy(n, nt, mask, coef, s);
        for (int32_t done = 0; done < max_sweeps && !converged[r]; ++done) {
            const uint32_t sweep = (uint32_t)sweeps[r];
            int64_t F = 0;
            for (int32_t k = 0; k < n; ++k) {
                const int32_t i = order[k];
                const int64_t d = 2 * (int64_t)s[i] * dense_field(nt, mask, coef, s, i);
                if (d < 0 || (rule == 1 && d == 0 && oracle_bit(seed, (uint32_t)i, sweep, instance_id, (uint32_t)r))) {
                    s[i] = (int8_t)-s[i];
                    E += d;
                    ++F;
                }
            }
            sweeps[r] += 1;
            flips[r] += F;
            if (until_converged && F == 0) converged[r] = 1;
        }
        energy[r] = E;
        if (until_converged && !converged[r]) notconv = 1;
    }
    return notconv;
}

/* The pass-based search of oracle_fm on a dense instance. */
int oracle_dense_fm(int32_t n, int64_t nt, const uint64_t* mask, const int64_t* coef, uint32_t instance_id,
                    int32_t restarts, uint64_t seed, int32_t max_passes, int32_t until_converged, int32_t init,
                    int8_t* spins, int64_t* energy, int64_t* passes, int64_t* kept, int8_t* converged)
{
    if (n < 1 || n > 64 || restarts < 1 || max_passes < 0) return -1;
    int notconv = 0;
    for (int32_t r = 0; r < restarts; ++r) {
        int8_t* s = spins + (int64_t)r * n;
        int8_t locked[64], best[64];
        if (init) {
            for (int32_t i = 0; i < n; ++i)
                s[i] = oracle_bit(seed, (uint32_t)i, 0xFFFFFFFFu, instance_id, (uint32_t)r) ? -1 : 1;
            passes[r] = 0;
            kept[r] = 0;
            converged[r] = 0;
        }
        int64_t E = oracle_dense_energy(n, nt, mask, coef, s);
        for (int32_t done = 0; done < max_passes && !converged[r]; ++done) {
            const int64_t E_start = E;
            int64_t E_cur = E, E_low = E, best_len = 0;
            memcpy(best, s, (size_t)n);
            memset(locked, 0, sizeof locked);
            for (int32_t step = 0; step < n; ++step) {
                int32_t pick = -1;
                int64_t pg = 0;
                for (int32_t i = 0; i < n; ++i) {
                    if (locked[i]) continue;
                    const int64_t g = -2 * (int64_t)s[i] * dense_field(nt, mask, coef, s, i);
                    if (pick < 0 || g > pg) {
                        pick = i;
                        pg = g;
                    }
                }
                s[pick] = (int8_t)-s[pick];
                locked[pick] = 1;
                E_cur -= pg;
                if (E_cur < E_low) {
                    E_low = E_cur;
                    best_len = step + 1;
                    memcpy(best, s, (size_t)n);
                }
            }
            memcpy(s, best, (size_t)n);
            E = E_low;
            passes[r] += 1;
            kept[r] += best_len;
            if (until_converged && !(E_low < E_start)) converged[r] = 1;
        }
        energy[r] = E;
        if (until_converged && !converged[r]) notconv = 1;
    }
    return notconv;
}

/* Exhaustive minimum over all 2^n states (n <= 30): returns E_min, writes one
 * minimising state and the number of minimising states. */
int64_t oracle_dense_brute(int32_t n, int64_t nt, const uint64_t* mask, const int64_t* coef, int8_t* best,
                           int64_t* count)
{
    if (n < 1 || n > 30) return INT64_MIN;
    int8_t s[64];
    int64_t Emin = INT64_MAX, cnt = 0;
    for (uint64_t code = 0; code < ((uint64_t)1 << n); ++code) {
        for (int i = 0; i < n; ++i) s[i] = ((code >> i) & 1u) ? -1 : 1;
        const int64_t E = oracle_dense_energy(n, nt, mask, coef, s);
        if (E < Emin) {
            Emin = E;
            cnt = 1;
            memcpy(best, s, (size_t)n);
        } else if (E == Emin) {
            ++cnt;
        }
    }
    *count = cnt;
    return Emin;
}

/* Best restart of one instance: lowest energy, lowest restart index on ties. */
int32_t oracle_best(int32_t restarts, const int64_t* energy, int64_t* best_E)
{
    int32_t b = 0;
    for (int32_t r = 1; r < restarts; ++r)
        if (energy[r] < energy[b]) b = r;
    if (best_E) *best_E = energy[b];
    return b;
}
