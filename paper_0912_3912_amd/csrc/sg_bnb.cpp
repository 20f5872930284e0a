// sg_bnb.cpp -- exact ground states by branch-and-bound (Sec. III), on the
// host CPU, seeded with a known state (for instance the best restart of the
// GPU descent) as the initial bound.
//
// Spins are assigned one at a time in breadth-first order of the primal
// graph (edges and the pairs of every triple) from spin 0, so that the
// neighbourhoods of early spins close early.  The bound of a partial
// assignment is the lower bound eq. (2), -sum|J| - sum|h| - sum|K|, raised by
// 2|c| for every term (field, coupling, triple) whose members are all assigned
// and whose contribution -c prod s is positive (eqs. (3)-(4), extended to the
// triples as Sec. VI does); at a leaf it is the energy.  Three prunes:
//   bound      the bound reaches the best energy found so far (a state of
//              that energy is already held);
//   dominance  a spin whose whole neighbourhood is assigned (the set F_s of
//              Lemma 1) would lower the energy by flipping (Lemma 2 with
//              one-spin changes);
//   tie        such a spin would leave the energy unchanged and holds the
//              value tried second: the same configuration with its first
//              value lies in a subtree searched before.
// The value of a spin tried first is its value in the seed state.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "sg.h"

namespace {

struct Term {
    int32_t a, b, c;  // members (-1 = absent); a is always present
    int32_t coef;
};

}  // namespace

// Defined in sg_host.cpp: the library's error reporting and validation.
sg_status sg_internal_fail(sg_status code, const char* msg);
sg_status sg_internal_validate(const sg_instance_desc* d);

extern "C" sg_status sg_exact_ground_state(const sg_instance_desc* d, const int8_t* seed_spins, int8_t* spins_out,
                                           int64_t* E_out, int64_t* nodes_out, int64_t max_nodes)
{
    if (!d || !spins_out || !E_out) return sg_internal_fail(SG_EINVAL, "sg_exact_ground_state: null argument");
    sg_status vs = sg_internal_validate(d);
    if (vs != SG_OK) return vs;
    const int32_t n = d->n;
    if (n > 4096) return sg_internal_fail(SG_EINVAL, "sg_exact_ground_state: at most 4096 spins");
    // terms and primal adjacency
    std::vector<Term> terms;
    std::vector<std::vector<int32_t>> adj((size_t)n);
    if (d->h)
        for (int32_t i = 0; i < n; ++i)
            if (d->h[i]) terms.push_back({i, -1, -1, d->h[i]});
    for (int64_t k = 0; k < d->m; ++k) {
        terms.push_back({d->ei[k], d->ej[k], -1, d->J[k]});
        adj[d->ei[k]].push_back(d->ej[k]);
        adj[d->ej[k]].push_back(d->ei[k]);
    }
    for (int64_t k = 0; k < d->t; ++k) {
        const int32_t a = d->tri[3 * k], b = d->tri[3 * k + 1], c = d->tri[3 * k + 2];
        terms.push_back({a, b, c, d->K[k]});
        adj[a].push_back(b); adj[a].push_back(c);
        adj[b].push_back(a); adj[b].push_back(c);
        adj[c].push_back(a); adj[c].push_back(b);
    }
    // breadth-first order over every component
    std::vector<int32_t> order, pos((size_t)n, -1);
    order.reserve((size_t)n);
    for (int32_t s0 = 0; s0 < n; ++s0) {
        if (pos[s0] >= 0) continue;
        pos[s0] = (int32_t)order.size();
        order.push_back(s0);
        for (size_t q = order.size() - 1; q < order.size(); ++q) {
            std::vector<int32_t> nb = adj[order[q]];
            std::sort(nb.begin(), nb.end());
            for (int32_t j : nb)
                if (pos[j] < 0) {
                    pos[j] = (int32_t)order.size();
                    order.push_back(j);
                }
        }
    }
    // terms closed at each depth; spins whose neighbourhood closes at each depth
    std::vector<std::vector<int32_t>> closes((size_t)n), settles((size_t)n);
    int64_t lb0 = 0;
    for (size_t t = 0; t < terms.size(); ++t) {
        const Term& T = terms[t];
        int32_t last = pos[T.a];
        if (T.b >= 0) last = std::max(last, pos[T.b]);
        if (T.c >= 0) last = std::max(last, pos[T.c]);
        closes[(size_t)last].push_back((int32_t)t);
        lb0 -= std::llabs((long long)T.coef);
    }
    std::vector<std::vector<int32_t>> term_of((size_t)n);  // terms of each spin (dominance tests)
    for (size_t t = 0; t < terms.size(); ++t) {
        term_of[terms[t].a].push_back((int32_t)t);
        if (terms[t].b >= 0) term_of[terms[t].b].push_back((int32_t)t);
        if (terms[t].c >= 0) term_of[terms[t].c].push_back((int32_t)t);
    }
    for (int32_t i = 0; i < n; ++i) {
        int32_t last = pos[i];
        for (int32_t j : adj[i]) last = std::max(last, pos[j]);
        settles[(size_t)last].push_back(i);
    }
    std::vector<int8_t> s((size_t)n, 0), first((size_t)n, 1), best((size_t)n, 1);
    int64_t bestE = INT64_MAX;
    auto energy_of = [&](const std::vector<int8_t>& v) {
        int64_t E = 0;
        for (const Term& T : terms) {
            int64_t p = v[T.a];
            if (T.b >= 0) p *= v[T.b];
            if (T.c >= 0) p *= v[T.c];
            E -= (int64_t)T.coef * p;
        }
        return E;
    };
    if (seed_spins) {
        for (int32_t i = 0; i < n; ++i) {
            if (seed_spins[i] != 1 && seed_spins[i] != -1)
                return sg_internal_fail(SG_EINVAL, "sg_exact_ground_state: seed spins must be +1 or -1");
            best[i] = first[i] = seed_spins[i];
        }
        bestE = energy_of(best);
    }
    auto term_value = [&](const Term& T) {  // -coef * prod s over assigned members
        int64_t p = s[T.a];
        if (T.b >= 0) p *= s[T.b];
        if (T.c >= 0) p *= s[T.c];
        return -(int64_t)T.coef * p;
    };
    // depth-first search; tried[k] = values tried at depth k (0, 1 or 2)
    std::vector<int8_t> tried((size_t)n, 0);
    std::vector<int64_t> lb_at((size_t)n + 1, 0);
    lb_at[0] = lb0;
    int64_t nodes = 0;
    bool budget_hit = false;
    int32_t k = 0;
    while (k >= 0) {
        if (tried[k] == 2) {  // both values done: unassign and go up
            tried[k] = 0;
            s[order[k]] = 0;
            --k;
            continue;
        }
        const int32_t i = order[k];
        s[i] = (int8_t)(tried[k] == 0 ? first[i] : -first[i]);
        ++tried[k];
        if (max_nodes > 0 && nodes >= max_nodes) {
            budget_hit = true;
            break;
        }
        ++nodes;
        int64_t lb = lb_at[k];
        for (int32_t t : closes[k]) lb += term_value(terms[t]) + std::llabs((long long)terms[t].coef);
        if (lb >= bestE) continue;  // bound
        bool pruned = false;
        for (int32_t j : settles[k]) {  // every term of j is now fully assigned
            int64_t f2 = 0;             // dE of flipping j = 2 * sum of its terms' values ... sign-flipped
            for (int32_t t : term_of[j]) f2 += term_value(terms[t]);
            // flipping j negates every term holding j: dE = -2 * sum(term values)
            const int64_t dE = -2 * f2;
            if (dE < 0) {
                pruned = true;
                break;
            }
            if (dE == 0 && s[j] != first[j]) {
                pruned = true;
                break;
            }
        }
        if (pruned) continue;
        if (k == n - 1) {  // leaf: lb is the energy
            bestE = lb;
            for (int32_t q = 0; q < n; ++q) best[q] = s[q];
            continue;
        }
        lb_at[k + 1] = lb;
        ++k;
    }
    for (int32_t i = 0; i < n; ++i) spins_out[i] = best[i];
    *E_out = bestE;
    if (nodes_out) *nodes_out = nodes;
    if (budget_hit) return sg_internal_fail(SG_ENOTCONV, "sg_exact_ground_state: node budget reached before proof");
    return SG_OK;
}
