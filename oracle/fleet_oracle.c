/*
 * fleet_oracle.c -- plain CPU oracle for the constrained scheduling model of
 * Tassone & Choudhury, "Algorithms for Optimizing Fleet Scheduling of Air
 * Ambulances" (arXiv 2002.11710), and for the paper's own forms of its three
 * algorithms.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table
 * or helper with the HIP implementation, nor with atabu_oracle.c (the oracle
 * of the unconstrained best-move search): the tests pin the two against each
 * other where their models coincide.
 *
 * The model (Section 3):
 *   - two travel-time matrices, one per vehicle type (Eq (1) at the
 *     helicopter speed and at the plane speed); vehicle v flies with the
 *     matrix of its type (b_k: 0 helicopter, 1 plane), Eq (2) sums each
 *     route's flights in that matrix;
 *   - mission n carries a time w_n by which its vehicle must arrive at its
 *     delivery point, and the vehicle then waits until w_n before it flies on
 *     (Eqs (8)-(9)); a vehicle leaves its base at time 0 and must be back by
 *     the horizon (24 h);
 *   - a route's flight time (waiting excluded) is at most the flight limit p
 *     (Eq (7));
 *   - a helicopter-only mission (f_n = 0) may not be flown by a plane (Eq (10)).
 *
 * What each function follows:
 *   fo_route_ok      a route's feasibility by definition: fly it, wait where
 *                    the model says so, check every arrival, the return and the
 *                    flight time.
 *   fo_keys          Algorithm 3 in the best-move form with these constraints:
 *                    every relocate and swap is scored, a move whose result is
 *                    infeasible is not a move; tabu moves are masked unless
 *                    they beat the best objective.  Mode 0 decides feasibility
 *                    and the cost change by applying the move to a copy and
 *                    checking both routes again; mode 1 from the edges the
 *                    move creates (each edge's check depends only on its two
 *                    ends, because a vehicle always leaves a mission at w_n).
 *   fo_greedy        Algorithm 1: helicopter-only missions first, each group
 *                    in order of the time limit, each mission appended to the
 *                    vehicle where it fits at the least added flight time;
 *                    when it fits nowhere, one sweep of Algorithm 2 over the
 *                    missions placed so far, then one more try; else an error.
 *   fo_solve_best    fo_greedy, then the best-move search (Tabu or NS).
 *   fo_solve_sweep   fo_greedy, then Algorithm 2 or 3 as printed: bases in
 *                    turn, each base's missions in turn, each mission moved to
 *                    the best strictly better place in another base;
 *                    TabuList entries with counters; passes until a pass moves
 *                    nothing.
 * The readings taken where the paper is silent or ambiguous are restated
 * where they are used.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FO_OK 0
#define FO_EINVAL (-1)
#define FO_ENOMEM (-3)
#define FO_EINFEAS (-6)   /* Algorithm 1 found no feasible start */

typedef struct {
    int32_t L;
    const int32_t *T[2];    /* T[0]: helicopter times, T[1]: plane times, L*L each */
    int32_t M;
    const int32_t *p, *d;   /* pickup, delivery locations */
    const int32_t *w;       /* time limit at the delivery point, seconds after the start;
                               NULL: no time limits and no horizon (Eqs (8)-(9) dropped) */
    const int32_t *heli;    /* 1: helicopter-only mission (f_n = 0); NULL: none */
    int32_t V;
    const int32_t *b;       /* base location */
    const int32_t *type;    /* 0 helicopter, 1 plane */
    int32_t flight_limit;   /* p, seconds of flight per vehicle (INT32_MAX: no limit) */
    int32_t horizon;        /* every vehicle back at its base by then */
} fo_inst;

typedef struct {
    int32_t variant;        /* 0 Tabu, 1 neighbourhood search */
    int32_t tenure;
    int32_t max_iters;      /* best-move: iterations; sweep: mission visits */
    int32_t aspiration;     /* best-move form only */
    uint64_t restart_seed;
} fo_params;

/* ------------------------------------------------------------------------ */
/* Routes                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t V, M;
    int32_t *len;   /* V */
    int32_t *r;     /* V*M, route v at r[v*M ..] */
} fsol;

static int fs_alloc(fsol *s, int32_t V, int32_t M)
{
    s->V = V; s->M = M;
    s->len = (int32_t *)calloc((size_t)V, sizeof(int32_t));
    s->r = (int32_t *)calloc((size_t)V * (size_t)(M > 0 ? M : 1), sizeof(int32_t));
    return (s->len && s->r) ? 0 : -1;
}

static void fs_free(fsol *s) { free(s->len); free(s->r); }

static void fs_copy(fsol *dst, const fsol *src)
{
    memcpy(dst->len, src->len, sizeof(int32_t) * (size_t)src->V);
    memcpy(dst->r, src->r, sizeof(int32_t) * (size_t)src->V * (size_t)(src->M > 0 ? src->M : 1));
}

static void fs_to_flat(const fsol *s, int32_t *off, int32_t *seq)
{
    int32_t o = 0;
    for (int32_t v = 0; v < s->V; ++v) {
        off[v] = o;
        for (int32_t k = 0; k < s->len[v]; ++k) seq[o++] = s->r[(int64_t)v * s->M + k];
    }
    off[s->V] = o;
}

static void fs_from_flat(fsol *s, const int32_t *off, const int32_t *seq)
{
    for (int32_t v = 0; v < s->V; ++v) {
        s->len[v] = off[v + 1] - off[v];
        for (int32_t k = 0; k < s->len[v]; ++k) s->r[(int64_t)v * s->M + k] = seq[off[v] + k];
    }
}

/* travel time from location x to location y for vehicle v */
static int64_t tv(const fo_inst *in, int32_t v, int32_t x, int32_t y)
{
    return in->T[in->type[v]][(int64_t)x * in->L + y];
}

static int32_t at(const fsol *s, int32_t v, int32_t k) { return s->r[(int64_t)v * s->M + k]; }

/* Eq (2) for one vehicle in its own matrix. */
static int64_t fo_route_cost(const fo_inst *in, const fsol *s, int32_t v)
{
    int32_t n = s->len[v];
    if (n == 0) return 0;
    int64_t c = tv(in, v, in->b[v], in->p[at(s, v, 0)]);
    for (int32_t k = 0; k < n; ++k) {
        int32_t m = at(s, v, k);
        c += tv(in, v, in->p[m], in->d[m]);
        if (k + 1 < n) c += tv(in, v, in->d[m], in->p[at(s, v, k + 1)]);
    }
    return c + tv(in, v, in->d[at(s, v, n - 1)], in->b[v]);
}

static int64_t fo_objective(const fo_inst *in, const fsol *s)
{
    int64_t c = 0;
    for (int32_t v = 0; v < in->V; ++v) c += fo_route_cost(in, s, v);
    return c;
}

/* Eqs (7)-(10) for one route, by definition: the vehicle leaves its base at
 * time 0, reaches each delivery no later than its time limit, waits there
 * until the limit, is back at its base by the horizon, flies at most the
 * flight limit, and carries no helicopter-only mission if it is a plane. */
static int fo_route_ok(const fo_inst *in, const fsol *s, int32_t v)
{
    int32_t n = s->len[v];
    if (n == 0) return 1;
    int64_t clock = 0;
    int32_t here = in->b[v];
    for (int32_t k = 0; k < n; ++k) {
        int32_t m = at(s, v, k);
        if (in->heli && in->heli[m] && in->type[v] != 0) return 0;
        if (in->w) {
            int64_t arrive = clock + tv(in, v, here, in->p[m]) + tv(in, v, in->p[m], in->d[m]);
            if (arrive > in->w[m]) return 0;
            clock = in->w[m];               /* wait until the mission's time limit */
        }
        here = in->d[m];
    }
    if (in->w && clock + tv(in, v, here, in->b[v]) > in->horizon) return 0;
    return fo_route_cost(in, s, v) <= in->flight_limit;
}

static int fo_solution_ok(const fo_inst *in, const fsol *s)
{
    for (int32_t v = 0; v < in->V; ++v)
        if (!fo_route_ok(in, s, v)) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Moves: the canonical numbering of the best-move search (relocate m into   */
/* global gap G = (missions before v) + v + g, index m*(M+V) + G; swap a < b, */
/* index M*(M+V) + a*M - a*(a+1)/2 + (b-a-1)), gaps counted before removal.  */
/* ------------------------------------------------------------------------ */
typedef struct { int swap; int32_t m, v, g, m1, m2; } fmove;

static void fo_locate(const fsol *s, int32_t m, int32_t *v, int32_t *k)
{
    for (int32_t u = 0; u < s->V; ++u)
        for (int32_t q = 0; q < s->len[u]; ++q)
            if (at(s, u, q) == m) { *v = u; *k = q; return; }
    *v = -1; *k = -1;
}

static int64_t fo_slots(int32_t M, int32_t V) { return (int64_t)M * (M + V) + (int64_t)M * (M - 1) / 2; }

/* 0 when the slot is a no-op */
static int fo_decode(const fo_inst *in, const fsol *s, int64_t idx, fmove *mv)
{
    int32_t M = in->M, V = in->V;
    int64_t R = (int64_t)M * (M + V);
    memset(mv, 0, sizeof(*mv));
    if (idx < R) {
        int32_t m = (int32_t)(idx / (M + V)), G = (int32_t)(idx % (M + V));
        int32_t before = 0, v;
        for (v = 0; v < V; ++v) {
            if (G >= before + v && G <= before + v + s->len[v]) break;
            before += s->len[v];
        }
        mv->m = m; mv->v = v; mv->g = G - before - v;
        int32_t sv, sk;
        fo_locate(s, m, &sv, &sk);
        return !(sv == v && (mv->g == sk || mv->g == sk + 1));
    }
    int64_t r = idx - R;
    int32_t a = 0;
    while (a + 1 < M && ((int64_t)(a + 1) * M - (int64_t)(a + 1) * (a + 2) / 2) <= r) ++a;
    mv->swap = 1;
    mv->m1 = a;
    mv->m2 = (int32_t)(a + 1 + (r - ((int64_t)a * M - (int64_t)a * (a + 1) / 2)));
    return 1;
}

static void fo_apply(fsol *s, const fmove *mv)
{
    int32_t M = s->M;
    if (!mv->swap) {
        int32_t sv, sk;
        fo_locate(s, mv->m, &sv, &sk);
        int32_t g = mv->g;
        if (sv == mv->v && g > sk) g -= 1;
        int32_t *src = s->r + (int64_t)sv * M;
        for (int32_t k = sk; k + 1 < s->len[sv]; ++k) src[k] = src[k + 1];
        s->len[sv] -= 1;
        int32_t *dst = s->r + (int64_t)mv->v * M;
        for (int32_t k = s->len[mv->v]; k > g; --k) dst[k] = dst[k - 1];
        dst[g] = mv->m;
        s->len[mv->v] += 1;
    } else {
        int32_t v1, k1, v2, k2;
        fo_locate(s, mv->m1, &v1, &k1);
        fo_locate(s, mv->m2, &v2, &k2);
        s->r[(int64_t)v1 * M + k1] = mv->m2;
        s->r[(int64_t)v2 * M + k2] = mv->m1;
    }
}

/* By definition: apply to a copy, check the routes the move touches, and
 * recompute Eq (2).  Returns 1 and the change if the result is feasible. */
static int fo_eval_def(const fo_inst *in, const fsol *s, fsol *tmp, const fmove *mv, int64_t *delta)
{
    fs_copy(tmp, s);
    fo_apply(tmp, mv);
    if (!fo_solution_ok(in, tmp)) return 0;
    *delta = fo_objective(in, tmp) - fo_objective(in, s);
    return 1;
}

/* ---- the same from the edges a move creates ------------------------------ */
/* A node of a route is a mission or the vehicle's base at either end.  With
 * the vehicle leaving mission n at w_n (and its base at 0), the flight x -> y
 * on vehicle v is feasible on its own terms: when y is a mission, leaving x
 * plus the flight to y's pickup and y's loaded leg reaches y's delivery by
 * w_y; when y is the base, leaving x plus the flight home is within the
 * horizon. */
typedef struct { int32_t exitl, enterl; int64_t leave; int32_t m; } fnode;   /* m = -1: base */

static fnode node_at(const fo_inst *in, const fsol *s, int32_t v, int32_t k)
{
    fnode x;
    if (k < 0 || k >= s->len[v]) { x.exitl = x.enterl = in->b[v]; x.leave = 0; x.m = -1; return x; }
    int32_t m = at(s, v, k);
    x.exitl = in->d[m]; x.enterl = in->p[m]; x.leave = in->w ? in->w[m] : 0; x.m = m;
    return x;
}

static fnode node_m(const fo_inst *in, int32_t m)
{
    fnode x = {in->d[m], in->p[m], in->w ? in->w[m] : 0, m};
    return x;
}

static int edge_ok(const fo_inst *in, int32_t v, fnode x, fnode y)
{
    if (!in->w) return 1;
    if (y.m < 0) return x.leave + tv(in, v, x.exitl, y.enterl) <= in->horizon;
    return x.leave + tv(in, v, x.exitl, y.enterl) + tv(in, v, in->p[y.m], in->d[y.m]) <= in->w[y.m];
}

/* flight x -> y on v (loaded leg of y included when y is a mission) */
static int64_t leg(const fo_inst *in, int32_t v, fnode x, fnode y)
{
    int64_t c = tv(in, v, x.exitl, y.enterl);
    if (y.m >= 0) c += tv(in, v, in->p[y.m], in->d[y.m]);
    return c;
}

static int compat(const fo_inst *in, int32_t m, int32_t v) { return !(in->heli && in->heli[m] && in->type[v] != 0); }

/* Incremental evaluation: 1 and the change if feasible.  cost[v] is each
 * route's current flight time. */
static int fo_eval_inc(const fo_inst *in, const fsol *s, const int32_t *rof, const int32_t *pof,
                       const int64_t *cost, const fmove *mv, int64_t *delta)
{
    if (!mv->swap) {
        int32_t m = mv->m, sv = rof[m], sk = pof[m], v = mv->v, g = mv->g;
        if (!compat(in, m, v)) return 0;
        fnode P = node_at(in, s, sv, sk - 1), N = node_at(in, s, sv, sk + 1), X = node_m(in, m);
        fnode A = node_at(in, s, v, g - 1), B = node_at(in, s, v, g);
        int64_t rem = leg(in, sv, P, N) - leg(in, sv, P, X) - leg(in, sv, X, N);
        int64_t ins = leg(in, v, A, X) + leg(in, v, X, B) - leg(in, v, A, B);
        if (!edge_ok(in, sv, P, N) || !edge_ok(in, v, A, X) || !edge_ok(in, v, X, B)) return 0;
        if (sv == v) {
            if (cost[v] + rem + ins > in->flight_limit) return 0;
        } else {
            if (cost[sv] + rem > in->flight_limit || cost[v] + ins > in->flight_limit) return 0;
        }
        *delta = rem + ins;
        return 1;
    }
    int32_t m1 = mv->m1, m2 = mv->m2;
    int32_t v1 = rof[m1], k1 = pof[m1], v2 = rof[m2], k2 = pof[m2];
    if (!compat(in, m2, v1) || !compat(in, m1, v2)) return 0;
    fnode X1 = node_m(in, m1), X2 = node_m(in, m2);
    if (v1 == v2 && (k2 == k1 + 1 || k1 == k2 + 1)) {
        fnode F = k1 < k2 ? X1 : X2, S = k1 < k2 ? X2 : X1;   /* F directly before S */
        int32_t kf = k1 < k2 ? k1 : k2;
        fnode P = node_at(in, s, v1, kf - 1), N = node_at(in, s, v1, kf + 2);
        if (!edge_ok(in, v1, P, S) || !edge_ok(in, v1, S, F) || !edge_ok(in, v1, F, N)) return 0;
        int64_t d = leg(in, v1, P, S) + leg(in, v1, S, F) + leg(in, v1, F, N)
                  - leg(in, v1, P, F) - leg(in, v1, F, S) - leg(in, v1, S, N);
        if (cost[v1] + d > in->flight_limit) return 0;
        *delta = d;
        return 1;
    }
    fnode P1 = node_at(in, s, v1, k1 - 1), N1 = node_at(in, s, v1, k1 + 1);
    fnode P2 = node_at(in, s, v2, k2 - 1), N2 = node_at(in, s, v2, k2 + 1);
    if (!edge_ok(in, v1, P1, X2) || !edge_ok(in, v1, X2, N1) ||
        !edge_ok(in, v2, P2, X1) || !edge_ok(in, v2, X1, N2)) return 0;
    int64_t d1 = leg(in, v1, P1, X2) + leg(in, v1, X2, N1) - leg(in, v1, P1, X1) - leg(in, v1, X1, N1);
    int64_t d2 = leg(in, v2, P2, X1) + leg(in, v2, X1, N2) - leg(in, v2, P2, X2) - leg(in, v2, X2, N2);
    if (v1 == v2) {
        if (cost[v1] + d1 + d2 > in->flight_limit) return 0;
    } else if (cost[v1] + d1 > in->flight_limit || cost[v2] + d2 > in->flight_limit) {
        return 0;
    }
    *delta = d1 + d2;
    return 1;
}

static void fo_index(const fsol *s, int32_t *rof, int32_t *pof)
{
    for (int32_t v = 0; v < s->V; ++v)
        for (int32_t k = 0; k < s->len[v]; ++k) { rof[at(s, v, k)] = v; pof[at(s, v, k)] = k; }
}

static uint64_t fo_key(int blocked, int64_t delta, int64_t idx)
{
    return ((uint64_t)(blocked ? 1 : 0) << 63) | ((uint64_t)(uint32_t)(delta + (1LL << 30)) << 32)
         | (uint64_t)(uint32_t)idx;
}

typedef struct {
    const fo_inst *in;
    fsol s, tmp;
    int32_t *rof, *pof;
    int64_t *cost;
} fview;

static int fv_init(fview *w, const fo_inst *in)
{
    w->in = in;
    if (fs_alloc(&w->s, in->V, in->M) || fs_alloc(&w->tmp, in->V, in->M)) return -1;
    w->rof = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
    w->pof = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
    w->cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)in->V);
    return (w->rof && w->pof && w->cost) ? 0 : -1;
}

static void fv_free(fview *w)
{
    fs_free(&w->s); fs_free(&w->tmp); free(w->rof); free(w->pof); free(w->cost);
}

static void fv_refresh(fview *w)
{
    fo_index(&w->s, w->rof, w->pof);
    for (int32_t v = 0; v < w->in->V; ++v) w->cost[v] = fo_route_cost(w->in, &w->s, v);
}

/* Keys of every slot (mode 0 by definition, 1 incremental); returns the minimum.
 * tabu_until[m*V + v] >= t: mission m may not enter vehicle v at iteration t. */
static uint64_t fo_scan(fview *w, const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
                        int variant, int aspiration, int mode, uint64_t *keys)
{
    const fo_inst *in = w->in;
    int32_t M = in->M, V = in->V;
    int64_t n = fo_slots(M, V);
    uint64_t kmin = UINT64_MAX;
    for (int64_t idx = 0; idx < n; ++idx) {
        fmove mv;
        uint64_t key = UINT64_MAX;
        int64_t dl = 0;
        if (fo_decode(in, &w->s, idx, &mv)) {
            int ok = mode == 0 ? fo_eval_def(in, &w->s, &w->tmp, &mv, &dl)
                               : fo_eval_inc(in, &w->s, w->rof, w->pof, w->cost, &mv, &dl);
            if (ok) {
                int tabu = 0;
                if (variant == 0) {
                    if (!mv.swap) tabu = tabu_until[(int64_t)mv.m * V + mv.v] >= t;
                    else tabu = tabu_until[(int64_t)mv.m1 * V + w->rof[mv.m2]] >= t
                             || tabu_until[(int64_t)mv.m2 * V + w->rof[mv.m1]] >= t;
                }
                key = fo_key(tabu && !(aspiration && cur + dl < best), dl, idx);
            }
        }
        if (keys) keys[idx] = key;
        if (key < kmin) kmin = key;
    }
    return kmin;
}

static int fo_check(const fo_inst *in)
{
    if (in->L < 1 || in->M < 0 || in->V < 1) return FO_EINVAL;
    for (int32_t m = 0; m < in->M; ++m) {
        if (in->p[m] < 0 || in->p[m] >= in->L || in->d[m] < 0 || in->d[m] >= in->L) return FO_EINVAL;
        if (in->p[m] == in->d[m] || (in->w && in->w[m] < 0)) return FO_EINVAL;
    }
    for (int32_t v = 0; v < in->V; ++v)
        if (in->b[v] < 0 || in->b[v] >= in->L || in->type[v] < 0 || in->type[v] > 1) return FO_EINVAL;
    for (int k = 0; k < 2; ++k)
        for (int64_t q = 0; q < (int64_t)in->L * in->L; ++q)
            if (in->T[k][q] < 0 || in->T[k][q] >= (1 << 27)) return FO_EINVAL;
    return FO_OK;
}

/* Public: every slot's key for a flattened state (mode 0 or 1). */
int fo_keys(const fo_inst *in, const int32_t *off, const int32_t *seq, const int32_t *tabu_until,
            int32_t t, int64_t cur, int64_t best, int32_t variant, int32_t aspiration, int32_t mode,
            uint64_t *keys)
{
    int rc = fo_check(in);
    if (rc) return rc;
    fview w;
    if (fv_init(&w, in)) { fv_free(&w); return FO_ENOMEM; }
    fs_from_flat(&w.s, off, seq);
    fv_refresh(&w);
    fo_scan(&w, tabu_until, t, cur, best, variant, aspiration, mode, keys);
    fv_free(&w);
    return FO_OK;
}

/* Public: feasibility and objective of a flattened solution. */
int fo_feasible(const fo_inst *in, const int32_t *off, const int32_t *seq, int64_t *obj)
{
    fsol s;
    if (fs_alloc(&s, in->V, in->M)) return FO_ENOMEM;
    fs_from_flat(&s, off, seq);
    int ok = fo_solution_ok(in, &s);
    *obj = fo_objective(in, &s);
    fs_free(&s);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014) for the seeded orders.               */
/* ------------------------------------------------------------------------ */
static uint64_t fo_next(uint64_t *st)
{
    uint64_t z = (*st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Fisher-Yates over a[0..n): for i = n-1 down to 1, j = next() % (i+1). */
static void fo_shuffle(int32_t *a, int32_t n, uint64_t *st)
{
    for (int32_t i = n - 1; i >= 1; --i) {
        int32_t j = (int32_t)(fo_next(st) % (uint64_t)(i + 1));
        int32_t x = a[i]; a[i] = a[j]; a[j] = x;
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 / 3 as printed: one pass over the bases (loop i), each base's  */
/* missions (loop j); each mission goes to the best strictly better place in */
/* another base (loops k, l).                                                 */
/*                                                                            */
/* Readings: every gap of base k is a candidate place (including before its   */
/* first mission); the first of equal candidates in (k, l) order is kept      */
/* (the paper replaces CurrentMin only on a better result), which is the      */
/* smallest gap id; the mission leaves base i only when the flight that then  */
/* joins its neighbours is feasible and base i's flight time stays within the */
/* limit; Algorithm 3's TabuList holds (mission, base left) selections: a     */
/* listed (j, k) skips base k for mission j (lines 20-27), a selection is     */
/* added with its counter at `tenure` only when the mission moves (it moves   */
/* only on improvement), and every counter drops by one at the end of each   */
/* mission's turn (line 56), the new one included, so an entry blocks the     */
/* next tenure - 1 turns; with restart seed s != 0 the base order of every    */
/* pass and the mission order of every base's turn are Fisher-Yates orders  */
/* drawn in that sequence from one SplitMix64(s) stream (the permutation      */
/* vectors of Section 4.2); the missions of base i are those on it when its   */
/* turn begins.                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t *ttl;      /* M*V counters, 0 = not listed */
} ftabu;

/* One mission's turn: returns 1 and fills the move if it moved. */
static int sweep_turn(fview *w, int32_t j, const ftabu *tb, int use_tabu, fmove *out, int64_t *delta, int64_t *gid)
{
    const fo_inst *in = w->in;
    int32_t V = in->V, i = w->rof[j], kj = w->pof[j];
    fnode P = node_at(in, &w->s, i, kj - 1), N = node_at(in, &w->s, i, kj + 1), X = node_m(in, j);
    if (!edge_ok(in, i, P, N)) return 0;
    int64_t rem = leg(in, i, P, N) - leg(in, i, P, X) - leg(in, i, X, N);
    if (w->cost[i] + rem > in->flight_limit) return 0;
    int64_t bestd = 0;             /* CurrentMin starts at the mission's current place */
    int found = 0;
    int32_t before = 0;
    for (int32_t k = 0; k < V; before += w->s.len[k], ++k) {
        if (k == i) continue;                                   /* lines 10-12 */
        if (!compat(in, j, k)) continue;                        /* lines 13-15 */
        if (use_tabu && tb->ttl[(int64_t)j * V + k] > 0) continue;  /* lines 20-27 */
        for (int32_t g = 0; g <= w->s.len[k]; ++g) {
            fnode A = node_at(in, &w->s, k, g - 1), B = node_at(in, &w->s, k, g);
            int64_t ins = leg(in, k, A, X) + leg(in, k, X, B) - leg(in, k, A, B);
            if (w->cost[k] + ins > in->flight_limit) continue;   /* lines 18-20 */
            if (!edge_ok(in, k, A, X) || !edge_ok(in, k, X, B)) continue;   /* lines 21-36 */
            if (rem + ins < bestd) {
                bestd = rem + ins;
                found = 1;
                out->swap = 0; out->m = j; out->v = k; out->g = g;
                *gid = before + k + g;
            }
        }
    }
    *delta = bestd;
    return found;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: helicopter-only missions first (lines 6-42), then the others  */
/* (lines 43-77), each group in order of the time limit (ties: mission id, or */
/* the seeded order's rank when the restart seed is not 0); a mission goes at */
/* the end of the vehicle where it fits (compatible, reached by its limit,   */
/* home by the horizon, within the flight limit) at the least added flight   */
/* time, ties to the lowest vehicle.  Where it fits nowhere: an error if no   */
/* mission is placed yet; else one pass of Algorithm 2 (neighbourhood search  */
/* sweep, identity orders) over the missions placed so far and one more try; */
/* an error if it still fits nowhere.  *err_mission: the mission that failed.*/
/* ------------------------------------------------------------------------ */
static int sweep_pass(fview *w, int use_tabu, ftabu *tb, int32_t tenure, uint64_t *rng,
                      int32_t *steps, int32_t max_steps, uint32_t *tr_move, int32_t *tr_delta,
                      int64_t *tr_obj, int64_t *cur, int32_t *moved, int32_t *last_improve);

static int fo_greedy_sol(const fo_inst *in, uint64_t seed, fview *w, int32_t *err_mission, int32_t *repairs)
{
    int32_t M = in->M, V = in->V;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t *placed = (int32_t *)calloc((size_t)(M + 1), sizeof(int32_t));
    for (int32_t i = 0; i < M; ++i) ord[i] = i;
    if (seed != 0) { uint64_t st = seed; fo_shuffle(ord, M, &st); }
    for (int32_t i = 0; i < M; ++i) rank[ord[i]] = i;
    /* order: helicopter-only first, then by time limit, then by rank (insertion sort: plain) */
    for (int32_t i = 0; i < M; ++i) ord[i] = i;
    for (int32_t i = 1; i < M; ++i) {
        int32_t x = ord[i], k = i - 1;
        while (k >= 0) {
            int32_t y = ord[k];
            int hx = in->heli ? in->heli[x] : 0, hy = in->heli ? in->heli[y] : 0;
            int32_t wx = in->w ? in->w[x] : 0, wy = in->w ? in->w[y] : 0;
            int before = hx != hy ? hx > hy : wx != wy ? wx < wy : rank[x] < rank[y];
            if (!before) break;
            ord[k + 1] = y; --k;
        }
        ord[k + 1] = x;
    }
    for (int32_t v = 0; v < V; ++v) w->s.len[v] = 0;
    int rc = FO_OK;
    *repairs = 0;
    for (int32_t q = 0; q < M && rc == FO_OK; ++q) {
        int32_t m = ord[q];
        for (int attempt = 0; attempt < 2; ++attempt) {
            fv_refresh(w);
            int32_t bv = -1;
            int64_t bestadd = 0;
            fnode X = node_m(in, m), B = {in->b[0], in->b[0], 0, -1};
            for (int32_t v = 0; v < V; ++v) {
                if (!compat(in, m, v)) continue;
                fnode Lst = node_at(in, &w->s, v, w->s.len[v] - 1);
                B.exitl = B.enterl = in->b[v];
                if (!edge_ok(in, v, Lst, X) || !edge_ok(in, v, X, B)) continue;
                int64_t add = leg(in, v, Lst, X) + leg(in, v, X, B) - leg(in, v, Lst, B);
                if (w->cost[v] + add > in->flight_limit) continue;
                if (bv < 0 || add < bestadd) { bv = v; bestadd = add; }
            }
            if (bv >= 0) {
                w->s.r[(int64_t)bv * M + w->s.len[bv]] = m;
                w->s.len[bv] += 1;
                placed[m] = 1;
                break;
            }
            if (attempt == 1 || q == 0) { *err_mission = m; rc = FO_EINFEAS; break; }
            /* repair: one Algorithm 2 sweep over the missions placed so far */
            int32_t steps = 0, moved = 0, li = -1;
            int64_t c = fo_objective(in, &w->s);
            fv_refresh(w);
            sweep_pass(w, 0, NULL, 0, NULL, &steps, INT32_MAX, NULL, NULL, NULL, &c, &moved, &li);
            *repairs += 1;
        }
    }
    fv_refresh(w);
    free(rank); free(ord); free(placed);
    return rc;
}

/* One pass (see above); returns 1 if the step budget ran out. */
static int sweep_pass(fview *w, int use_tabu, ftabu *tb, int32_t tenure, uint64_t *rng,
                      int32_t *steps, int32_t max_steps, uint32_t *tr_move, int32_t *tr_delta,
                      int64_t *tr_obj, int64_t *cur, int32_t *moved, int32_t *last_improve)
{
    const fo_inst *in = w->in;
    int32_t M = in->M, V = in->V;
    int32_t *vord = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    int out_of_budget = 0;
    for (int32_t v = 0; v < V; ++v) vord[v] = v;
    if (rng) fo_shuffle(vord, V, rng);
    for (int32_t vi = 0; vi < V && !out_of_budget; ++vi) {
        int32_t i = vord[vi], n = w->s.len[i];
        for (int32_t k = 0; k < n; ++k) list[k] = at(&w->s, i, k);
        if (rng) fo_shuffle(list, n, rng);
        for (int32_t q = 0; q < n; ++q) {
            if (*steps >= max_steps) { out_of_budget = 1; break; }
            int32_t j = list[q];
            fmove mv;
            int64_t d = 0, gid = 0;
            int ok = sweep_turn(w, j, tb, use_tabu, &mv, &d, &gid);
            if (ok) {
                int32_t left = w->rof[j];
                fo_apply(&w->s, &mv);
                fv_refresh(w);
                *cur += d;
                *moved += 1;
                *last_improve = *steps;
                if (use_tabu) tb->ttl[(int64_t)j * V + left] = tenure;   /* line 55 */
            }
            if (tr_move) {
                tr_move[*steps] = ok ? (uint32_t)((int64_t)j * (M + V) + gid) : 0xFFFFFFFFu;
                tr_delta[*steps] = ok ? (int32_t)d : 0;
                tr_obj[*steps] = *cur;
            }
            if (use_tabu)                                               /* line 56 */
                for (int64_t e = 0; e < (int64_t)M * V; ++e)
                    if (tb->ttl[e] > 0) tb->ttl[e] -= 1;
            *steps += 1;
        }
    }
    free(vord); free(list);
    return out_of_budget;
}

/* Public: Algorithm 1 alone. */
int fo_greedy(const fo_inst *in, uint64_t seed, int32_t *off, int32_t *seq, int32_t *err_mission,
              int32_t *repairs)
{
    int rc = fo_check(in);
    if (rc) return rc;
    fview w;
    if (fv_init(&w, in)) { fv_free(&w); return FO_ENOMEM; }
    *err_mission = -1;
    rc = fo_greedy_sol(in, seed, &w, err_mission, repairs);
    if (rc == FO_OK) fs_to_flat(&w.s, off, seq);
    fv_free(&w);
    return rc;
}

/* Public: Algorithm 1, then the best-move search (Tabu or NS) with the
 * constraints.  Outputs as the unconstrained oracle's or_solve: best and final
 * routes, objectives, iterations, trace (bit0 swap, bit1 aspirated tabu move,
 * bit2 fallback). */
int fo_solve_best(const fo_inst *in, const fo_params *pr, int32_t *best_off, int32_t *best_seq,
                  int32_t *final_off, int32_t *final_seq, int64_t *best_obj, int64_t *final_obj,
                  int32_t *iters_done, int32_t *best_iter, uint32_t *tr_move, int32_t *tr_delta,
                  int64_t *tr_obj, uint8_t *tr_flags, int32_t *err_mission)
{
    int rc = fo_check(in);
    if (rc) return rc;
    if (pr->tenure < 0 || pr->max_iters < 0 || (pr->variant != 0 && pr->variant != 1)) return FO_EINVAL;
    int32_t M = in->M, V = in->V;
    fview w;
    if (fv_init(&w, in)) { fv_free(&w); return FO_ENOMEM; }
    int32_t repairs = 0;
    *err_mission = -1;
    rc = fo_greedy_sol(in, pr->restart_seed, &w, err_mission, &repairs);
    if (rc) { fv_free(&w); return rc; }
    int32_t *tabu = (int32_t *)malloc(sizeof(int32_t) * ((size_t)M * V + 1));
    for (int64_t e = 0; e < (int64_t)M * V; ++e) tabu[e] = -1;
    int64_t cur = fo_objective(in, &w.s), best = cur;
    int32_t bi = -1, done = 0;
    fs_to_flat(&w.s, best_off, best_seq);
    for (int32_t t = 0; t < pr->max_iters; ++t) {
        uint64_t k = fo_scan(&w, tabu, t, cur, best, pr->variant, pr->aspiration, 1, NULL);
        uint32_t move = 0xFFFFFFFFu;
        int32_t dl = 0;
        uint8_t fl = 0;
        if (k != UINT64_MAX) {
            int blocked = (int)(k >> 63);
            int64_t d = (int64_t)((k >> 32) & 0x7FFFFFFFu) - (1LL << 30);
            int64_t idx = (int64_t)(k & 0xFFFFFFFFu);
            if (pr->variant == 1 && d >= 0) break;              /* local optimum */
            fmove mv;
            fo_decode(in, &w.s, idx, &mv);
            int was_tabu = 0;
            if (pr->variant == 0) {
                if (!mv.swap) {
                    was_tabu = tabu[(int64_t)mv.m * V + mv.v] >= t;
                    tabu[(int64_t)mv.m * V + w.rof[mv.m]] = t + pr->tenure;
                } else {
                    int32_t r1 = w.rof[mv.m1], r2 = w.rof[mv.m2];
                    was_tabu = tabu[(int64_t)mv.m1 * V + r2] >= t || tabu[(int64_t)mv.m2 * V + r1] >= t;
                    tabu[(int64_t)mv.m1 * V + r1] = t + pr->tenure;
                    tabu[(int64_t)mv.m2 * V + r2] = t + pr->tenure;
                }
            }
            fo_apply(&w.s, &mv);
            fv_refresh(&w);
            cur += d;
            move = (uint32_t)idx; dl = (int32_t)d;
            fl = (uint8_t)((mv.swap ? 1 : 0) | ((was_tabu && !blocked) ? 2 : 0) | (blocked ? 4 : 0));
        } else if (pr->variant == 1) {
            break;
        }
        if (tr_move) { tr_move[t] = move; tr_delta[t] = dl; tr_obj[t] = cur; tr_flags[t] = fl; }
        done = t + 1;
        if (cur < best) { best = cur; bi = t; fs_to_flat(&w.s, best_off, best_seq); }
    }
    fs_to_flat(&w.s, final_off, final_seq);
    *best_obj = best; *final_obj = cur; *iters_done = done; *best_iter = bi;
    free(tabu);
    fv_free(&w);
    return FO_OK;
}

/* Public: Algorithm 1, then Algorithm 2 (variant 1) or 3 (variant 0) as
 * printed (see sweep_pass).  One trace record per mission turn: the relocate
 * slot index of the move in the best-move numbering (0xFFFFFFFF when the
 * mission stays), its change and the objective after it.  Passes run until
 * one moves nothing or max_iters turns have run; the objective only falls,
 * so the best solution is the final one. */
int fo_solve_sweep(const fo_inst *in, const fo_params *pr, int32_t *off, int32_t *seq,
                   int64_t *obj, int32_t *iters_done, int32_t *best_iter, int32_t *passes,
                   uint32_t *tr_move, int32_t *tr_delta, int64_t *tr_obj, int32_t *err_mission)
{
    int rc = fo_check(in);
    if (rc) return rc;
    if (pr->tenure < 0 || pr->max_iters < 0 || (pr->variant != 0 && pr->variant != 1)) return FO_EINVAL;
    int32_t M = in->M, V = in->V;
    fview w;
    if (fv_init(&w, in)) { fv_free(&w); return FO_ENOMEM; }
    int32_t repairs = 0;
    *err_mission = -1;
    rc = fo_greedy_sol(in, pr->restart_seed, &w, err_mission, &repairs);
    if (rc) { fv_free(&w); return rc; }
    ftabu tb;
    tb.ttl = (int32_t *)calloc((size_t)M * V + 1, sizeof(int32_t));
    uint64_t st = pr->restart_seed;
    int64_t cur = fo_objective(in, &w.s);
    int32_t steps = 0, np = 0, li = -1;
    for (;;) {
        int32_t moved = 0;
        int out = sweep_pass(&w, pr->variant == 0, &tb, pr->tenure, pr->restart_seed ? &st : NULL, &steps,
                             pr->max_iters, tr_move, tr_delta, tr_obj, &cur, &moved, &li);
        np += 1;
        if (out || moved == 0) break;
    }
    fs_to_flat(&w.s, off, seq);
    *obj = cur; *iters_done = steps; *best_iter = li; *passes = np;
    free(tb.ttl);
    fv_free(&w);
    return FO_OK;
}
