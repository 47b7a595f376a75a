/*
 * atabu_oracle.c -- plain CPU oracle for the Tabu-search / neighbourhood-search
 * scheduler of Tassone & Choudhury, "Algorithms for Optimizing Fleet Scheduling
 * of Air Ambulances" (arXiv 2002.11710).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the HIP implementation; it is written to be read against the
 * paper, not to be fast.
 *
 * What each function follows:
 *   or_travel      Eq (1): haversine distance divided by the vehicle speed,
 *                  in FP64, rounded to integer seconds.
 *   or_objective   Eq (2) specialised to route lists: total time flown, each
 *                  mission's loaded leg included, every route starting and
 *                  ending at its vehicle's base (Eqs (3)-(7) hold by
 *                  construction of the route lists).
 *   or_greedy      Algorithm 1 (scheduling initialisation) without its
 *                  feasibility checks: missions are taken in a fixed order
 *                  and appended after the previously assigned mission of the
 *                  vehicle with the least added time.
 *   or_delta_def   a move's cost change by definition: apply it to a copy and
 *                  recompute Eq (2) in full.
 *   or_delta_inc   the same change from the closed forms of the few edges a
 *                  relocate or swap move touches (Figure 2 shows a relocate).
 *   or_step        one iteration of Algorithm 3 (Tabu search) or Algorithm 2
 *                  (neighbourhood search) in the best-move form: score every
 *                  relocate and swap move, mask tabu moves unless they beat
 *                  the best objective found (aspiration), take the smallest
 *                  (delta, index) and apply it; the moved mission becomes tabu
 *                  for its old vehicle.
 *   or_solve       greedy start, then or_step for the iteration budget.
 *
 * Readings of points the paper leaves open are listed in the project's design
 * notes; the ones that change numbers are restated where they are used.
 *
 * Parity pins (tests/test_oracle_*.py): closed-form meridian distances and an
 * independent Python haversine for or_travel; a hand-computed one-mission
 * objective and an independent Python route sum for or_objective; brute-force
 * enumeration of every solution (and a Held-Karp subset DP) for the optimum
 * the search must not beat; or_delta_inc against or_delta_def on every move of
 * random solutions; route invariants after every step; the neighbourhood
 * search stopping only at a true local optimum.  SplitMix64 against the
 * generator's published reference outputs; the greedy start against a
 * hand-worked shuffled order, a hand-computed instance where the route's old
 * return leg decides the vehicle, and exact ties; each step's tabu writes
 * (exactly the moved missions' entries for the vehicles they left, at
 * t + tenure), the (mission, vehicle) entries that make a slot tabu, strict
 * aspiration, the trace flags, and the choice of the admissible move with the
 * smallest by-definition delta, ties to the smallest slot index.  A whole
 * trajectory is the composition of those pinned steps; the paper prints no
 * worked trajectory to compare one against.
 */
#define _GNU_SOURCE 1
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_ENOMEM (-3)

typedef struct {
    int32_t L;            /* locations */
    const int32_t *T;     /* L*L travel seconds, T[i*L + j] = time i -> j */
    int32_t M;            /* missions */
    const int32_t *p;     /* pickup location of each mission */
    const int32_t *d;     /* delivery location of each mission */
    int32_t V;            /* vehicles */
    const int32_t *b;     /* base location of each vehicle */
} or_inst;

typedef struct {
    int32_t variant;      /* 0 Tabu search, 1 neighbourhood search */
    int32_t tenure;
    int32_t max_iters;
    int32_t aspiration;   /* 1: a tabu move that beats the best objective is allowed */
    uint64_t restart_seed;
} or_params;

/* ------------------------------------------------------------------------ */
/* Eq (1): travel time between two points from the haversine formula.        */
/* Earth radius 6371 km; latitude/longitude in degrees; FP64 throughout;     */
/* the result in seconds rounded half away from zero.                        */
/* ------------------------------------------------------------------------ */
int or_travel(int32_t n, const double *lat_deg, const double *lon_deg,
              double speed_kmh, int32_t *out)
{
    if (n < 0 || !(speed_kmh > 0.0)) return OR_EINVAL;
    const double rad = M_PI / 180.0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < n; ++j) {
            double phi_i = lat_deg[i] * rad, phi_j = lat_deg[j] * rad;
            double psi_i = lon_deg[i] * rad, psi_j = lon_deg[j] * rad;
            double s1 = sin((phi_j - phi_i) / 2.0);
            double s2 = sin((psi_j - psi_i) / 2.0);
            double a = s1 * s1 + cos(phi_i) * cos(phi_j) * s2 * s2;
            double km = 2.0 * 6371.0 * asin(sqrt(fmin(1.0, a)));
            double sec = km * 3600.0 / speed_kmh;
            out[(int64_t)i * n + j] = (int32_t)llround(sec);
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Solutions as plain route lists.                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t V, M;
    int32_t *len;   /* V */
    int32_t *r;     /* V*M: route v is r[v*M .. v*M+len[v]) */
} sol_t;

static int sol_alloc(sol_t *s, int32_t V, int32_t M)
{
    s->V = V; s->M = M;
    s->len = (int32_t *)calloc((size_t)V, sizeof(int32_t));
    s->r = (int32_t *)calloc((size_t)V * (size_t)(M > 0 ? M : 1), sizeof(int32_t));
    return (s->len && s->r) ? 0 : -1;
}

static void sol_free(sol_t *s) { free(s->len); free(s->r); s->len = NULL; s->r = NULL; }

static void sol_copy(sol_t *dst, const sol_t *src)
{
    memcpy(dst->len, src->len, sizeof(int32_t) * (size_t)src->V);
    memcpy(dst->r, src->r, sizeof(int32_t) * (size_t)src->V * (size_t)(src->M > 0 ? src->M : 1));
}

static void sol_from_flat(sol_t *s, const int32_t *off, const int32_t *seq)
{
    for (int32_t v = 0; v < s->V; ++v) {
        s->len[v] = off[v + 1] - off[v];
        for (int32_t k = 0; k < s->len[v]; ++k) s->r[v * s->M + k] = seq[off[v] + k];
    }
}

static void sol_to_flat(const sol_t *s, int32_t *off, int32_t *seq)
{
    int32_t o = 0;
    for (int32_t v = 0; v < s->V; ++v) {
        off[v] = o;
        for (int32_t k = 0; k < s->len[v]; ++k) seq[o++] = s->r[v * s->M + k];
    }
    off[s->V] = o;
}

static int32_t TT(const or_inst *in, int32_t i, int32_t j) { return in->T[(int64_t)i * in->L + j]; }

/* Eq (2) for one vehicle: base -> pickup of the first mission, each mission's
 * loaded leg pickup -> delivery, delivery -> next pickup, last delivery ->
 * base.  An unused vehicle does not fly. */
static int64_t route_cost(const or_inst *in, const sol_t *s, int32_t v)
{
    int32_t n = s->len[v];
    if (n == 0) return 0;
    const int32_t *r = s->r + (int64_t)v * s->M;
    int32_t base = in->b[v];
    int64_t c = TT(in, base, in->p[r[0]]);
    for (int32_t k = 0; k < n; ++k) {
        c += TT(in, in->p[r[k]], in->d[r[k]]);
        if (k + 1 < n) c += TT(in, in->d[r[k]], in->p[r[k + 1]]);
    }
    c += TT(in, in->d[r[n - 1]], base);
    return c;
}

static int64_t sol_objective(const or_inst *in, const sol_t *s)
{
    int64_t c = 0;
    for (int32_t v = 0; v < s->V; ++v) c += route_cost(in, s, v);
    return c;
}

/* Where is mission m: vehicle and position. */
static void locate(const sol_t *s, int32_t m, int32_t *v_out, int32_t *k_out)
{
    for (int32_t v = 0; v < s->V; ++v)
        for (int32_t k = 0; k < s->len[v]; ++k)
            if (s->r[v * s->M + k] == m) { *v_out = v; *k_out = k; return; }
    *v_out = -1; *k_out = -1;
}

/* ------------------------------------------------------------------------ */
/* Moves and their canonical numbering.                                       */
/*                                                                            */
/* Relocate (Figure 2): take mission m out of its route and put it into gap g */
/* of vehicle v, where gap g of a route of n missions (g = 0..n) lies between */
/* its (g-1)-th mission (or the base when g = 0) and its g-th mission (or the */
/* base when g = n); gaps are numbered in the route BEFORE m is removed.      */
/* Gap ids run over all vehicles in order: G(v,g) = (missions on vehicles     */
/* before v) + v + g, so there are M+V gaps.  Relocate index = m*(M+V) + G.   */
/* The two gaps on either side of m in its own route leave the solution       */
/* unchanged and are not moves.                                               */
/*                                                                            */
/* Swap: missions m1 < m2 exchange places (any routes, adjacent or not).      */
/* Index = M*(M+V) + m1*M - m1*(m1+1)/2 + (m2 - m1 - 1).                      */
/* ------------------------------------------------------------------------ */
static int64_t n_slots(int32_t M, int32_t V)
{
    return (int64_t)M * (M + V) + (int64_t)M * (M - 1) / 2;
}

typedef struct {
    int is_swap;
    int32_t m, v, g;       /* relocate: mission, target vehicle, target gap */
    int32_t m1, m2;        /* swap */
} move_t;

/* Decode a slot index against solution s.  Returns 0 when the slot is not a move. */
static int decode(const or_inst *in, const sol_t *s, int64_t idx, move_t *mv)
{
    int32_t M = in->M, V = in->V;
    int64_t R = (int64_t)M * (M + V);
    memset(mv, 0, sizeof(*mv));
    if (idx < 0 || idx >= n_slots(M, V)) return 0;
    if (idx < R) {
        int32_t m = (int32_t)(idx / (M + V));
        int32_t G = (int32_t)(idx % (M + V));
        int32_t before = 0, v = 0;
        for (v = 0; v < V; ++v) {
            int32_t first = before + v, last = before + v + s->len[v];
            if (G >= first && G <= last) break;
            before += s->len[v];
        }
        int32_t g = G - before - v;
        mv->is_swap = 0; mv->m = m; mv->v = v; mv->g = g;
        int32_t mv_v, mv_k;
        locate(s, m, &mv_v, &mv_k);
        if (mv_v == v && (g == mv_k || g == mv_k + 1)) return 0;   /* no change */
        return 1;
    }
    int64_t r = idx - R;
    int32_t m1 = 0;
    while (m1 + 1 < M && ((int64_t)(m1 + 1) * M - (int64_t)(m1 + 1) * (m1 + 2) / 2) <= r) ++m1;
    int64_t base = (int64_t)m1 * M - (int64_t)m1 * (m1 + 1) / 2;
    mv->is_swap = 1; mv->m1 = m1; mv->m2 = (int32_t)(m1 + 1 + (r - base));
    return 1;
}

/* Apply a (valid) move to s by editing the route lists. */
static void apply_move(sol_t *s, const move_t *mv)
{
    int32_t M = s->M;
    if (!mv->is_swap) {
        int32_t sv, sk;
        locate(s, mv->m, &sv, &sk);
        int32_t g = mv->g;
        /* gap numbering is in the route before removal: a later gap of the same
         * route moves one place left once m is out */
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
        locate(s, mv->m1, &v1, &k1);
        locate(s, mv->m2, &v2, &k2);
        s->r[(int64_t)v1 * M + k1] = mv->m2;
        s->r[(int64_t)v2 * M + k2] = mv->m1;
    }
}

/* Cost change by definition: apply to a copy, recompute Eq (2), subtract. */
static int64_t delta_def(const or_inst *in, const sol_t *s, sol_t *scratch, const move_t *mv)
{
    sol_copy(scratch, s);
    apply_move(scratch, mv);
    return sol_objective(in, scratch) - sol_objective(in, s);
}

/* Exit location of a route element (a mission's delivery) and its entry
 * location (the pickup).  k = -1 or k = len stands for the vehicle's base. */
static int32_t exit_loc(const or_inst *in, const sol_t *s, int32_t v, int32_t k)
{
    if (k < 0 || k >= s->len[v]) return in->b[v];
    return in->d[s->r[(int64_t)v * s->M + k]];
}

static int32_t enter_loc(const or_inst *in, const sol_t *s, int32_t v, int32_t k)
{
    if (k < 0 || k >= s->len[v]) return in->b[v];
    return in->p[s->r[(int64_t)v * s->M + k]];
}

/* Cost change from the edges the move touches.  With t(x->y) the flight from
 * x's exit to y's entry and P, N a mission's neighbours (possibly the base):
 *   relocate m into gap (a,b):  [t(P->N) - t(P->m) - t(m->N)]
 *                               + [t(a->m) + t(m->b) - t(a->b)]
 *   swap, not adjacent:  each mission takes the other's two edges;
 *   swap, m1 directly before m2:  P1 m1 m2 N2  becomes  P1 m2 m1 N2.
 * The loaded legs (pickup -> delivery) are unchanged by every move.
 * route_of / pos_of give each mission's vehicle and position in s. */
static int64_t delta_inc(const or_inst *in, const sol_t *s, const int32_t *route_of,
                         const int32_t *pos_of, const move_t *mv)
{
    if (!mv->is_swap) {
        int32_t m = mv->m, sv = route_of[m], sk = pos_of[m];
        int32_t xP = exit_loc(in, s, sv, sk - 1), yN = enter_loc(in, s, sv, sk + 1);
        int64_t rem = (int64_t)TT(in, xP, yN) - TT(in, xP, in->p[m]) - TT(in, in->d[m], yN);
        int32_t xa = exit_loc(in, s, mv->v, mv->g - 1), yb = enter_loc(in, s, mv->v, mv->g);
        int64_t ins = (int64_t)TT(in, xa, in->p[m]) + TT(in, in->d[m], yb) - TT(in, xa, yb);
        return rem + ins;
    }
    int32_t m1 = mv->m1, m2 = mv->m2;
    int32_t v1 = route_of[m1], k1 = pos_of[m1], v2 = route_of[m2], k2 = pos_of[m2];
    if (v1 == v2 && (k2 == k1 + 1 || k1 == k2 + 1)) {
        int32_t a = m1, c = m2, ka = k1, kc = k2;
        if (k1 == k2 + 1) { a = m2; c = m1; ka = k2; kc = k1; }
        /* a directly before c */
        int32_t xP = exit_loc(in, s, v1, ka - 1), yN = enter_loc(in, s, v1, kc + 1);
        int64_t before = (int64_t)TT(in, xP, in->p[a]) + TT(in, in->d[a], in->p[c]) + TT(in, in->d[c], yN);
        int64_t after = (int64_t)TT(in, xP, in->p[c]) + TT(in, in->d[c], in->p[a]) + TT(in, in->d[a], yN);
        return after - before;
    }
    int32_t xP1 = exit_loc(in, s, v1, k1 - 1), yN1 = enter_loc(in, s, v1, k1 + 1);
    int32_t xP2 = exit_loc(in, s, v2, k2 - 1), yN2 = enter_loc(in, s, v2, k2 + 1);
    int64_t before = (int64_t)TT(in, xP1, in->p[m1]) + TT(in, in->d[m1], yN1)
                   + TT(in, xP2, in->p[m2]) + TT(in, in->d[m2], yN2);
    int64_t after = (int64_t)TT(in, xP1, in->p[m2]) + TT(in, in->d[m2], yN1)
                  + TT(in, xP2, in->p[m1]) + TT(in, in->d[m1], yN2);
    return after - before;
}

/* Vehicle and position of every mission in s. */
static void index_missions(const sol_t *s, int32_t *route_of, int32_t *pos_of)
{
    for (int32_t v = 0; v < s->V; ++v)
        for (int32_t k = 0; k < s->len[v]; ++k) {
            int32_t m = s->r[v * s->M + k];
            route_of[m] = v; pos_of[m] = k;
        }
}

/* ------------------------------------------------------------------------ */
/* Input checks shared by every entry point.                                  */
/* ------------------------------------------------------------------------ */
static int check_inst(const or_inst *in)
{
    if (in->L < 1 || in->M < 0 || in->V < 1) return OR_EINVAL;
    for (int32_t m = 0; m < in->M; ++m) {
        if (in->p[m] < 0 || in->p[m] >= in->L || in->d[m] < 0 || in->d[m] >= in->L) return OR_EINVAL;
        if (in->p[m] == in->d[m]) return OR_EINVAL;
    }
    for (int32_t v = 0; v < in->V; ++v)
        if (in->b[v] < 0 || in->b[v] >= in->L) return OR_EINVAL;
    /* the key packs delta + 2^30 into 31 bits; a delta sums at most three
     * travel times minus three others, so times below 2^27 (max T * 8 < 2^30)
     * keep every delta inside that field */
    for (int64_t k = 0; k < (int64_t)in->L * in->L; ++k)
        if (in->T[k] < 0 || in->T[k] >= (1 << 27)) return OR_ERANGE;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Public: objective of a flattened solution (off: V+1, seq: M).              */
/* ------------------------------------------------------------------------ */
int64_t or_objective(const or_inst *in, const int32_t *off, const int32_t *seq)
{
    sol_t s;
    if (sol_alloc(&s, in->V, in->M)) return -1;
    sol_from_flat(&s, off, seq);
    int64_t c = sol_objective(in, &s);
    sol_free(&s);
    return c;
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): golden-gamma increment,
 * then the 30/27/31 xor-shift-multiply finaliser. */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Public: the first n outputs of SplitMix64(seed) (pinned to the generator's
 * published reference outputs). */
void or_splitmix64(uint64_t seed, int32_t n, uint64_t *out)
{
    uint64_t st = seed;
    for (int32_t i = 0; i < n; ++i) out[i] = splitmix64_next(&st);
}

/* Algorithm 1, generalised (no deadlines, flight limit or vehicle types):
 * missions in order pi (identity for seed 0, else a Fisher-Yates shuffle
 * driven by SplitMix64(seed)); each is appended after the last mission of the
 * vehicle whose route time grows least, ties to the lowest vehicle. */
static void greedy(const or_inst *in, uint64_t seed, sol_t *s)
{
    int32_t M = in->M, V = in->V;
    int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M > 0 ? M : 1));
    for (int32_t i = 0; i < M; ++i) pi[i] = i;
    if (seed != 0) {
        uint64_t st = seed;
        for (int32_t i = M - 1; i >= 1; --i) {
            int32_t j = (int32_t)(splitmix64_next(&st) % (uint64_t)(i + 1));
            int32_t tmp = pi[i]; pi[i] = pi[j]; pi[j] = tmp;
        }
    }
    for (int32_t v = 0; v < V; ++v) s->len[v] = 0;
    for (int32_t i = 0; i < M; ++i) {
        int32_t m = pi[i];
        int64_t best = 0; int32_t bv = -1;
        for (int32_t v = 0; v < V; ++v) {
            int32_t last = s->len[v] == 0 ? in->b[v] : in->d[s->r[(int64_t)v * M + s->len[v] - 1]];
            int64_t add = (int64_t)TT(in, last, in->p[m]) + TT(in, in->p[m], in->d[m])
                        + TT(in, in->d[m], in->b[v]) - TT(in, last, in->b[v]);
            if (bv < 0 || add < best) { best = add; bv = v; }
        }
        s->r[(int64_t)bv * M + s->len[bv]] = m;
        s->len[bv] += 1;
    }
    free(pi);
}

int or_greedy(const or_inst *in, uint64_t seed, int32_t *off, int32_t *seq)
{
    int rc = check_inst(in);
    if (rc) return rc;
    sol_t s;
    if (sol_alloc(&s, in->V, in->M)) return OR_ENOMEM;
    greedy(in, seed, &s);
    sol_to_flat(&s, off, seq);
    sol_free(&s);
    return OR_OK;
}

/* Public: cost change of slot idx on a flattened solution, by definition
 * (mode 0) or from the closed forms (mode 1).  *valid = 0 for non-moves. */
int64_t or_delta(const or_inst *in, const int32_t *off, const int32_t *seq,
                 int64_t idx, int32_t mode, int32_t *valid)
{
    sol_t s, tmp;
    if (sol_alloc(&s, in->V, in->M)) return 0;
    if (sol_alloc(&tmp, in->V, in->M)) { sol_free(&s); return 0; }
    sol_from_flat(&s, off, seq);
    move_t mv;
    int64_t r = 0;
    *valid = decode(in, &s, idx, &mv);
    if (*valid) {
        if (mode == 0) {
            r = delta_def(in, &s, &tmp, &mv);
        } else {
            int32_t *ro = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
            int32_t *po = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
            index_missions(&s, ro, po);
            r = delta_inc(in, &s, ro, po, &mv);
            free(ro); free(po);
        }
    }
    sol_free(&s);
    sol_free(&tmp);
    return r;
}

/* Public: apply slot idx to a flattened solution in place. */
int or_apply(const or_inst *in, int32_t *off, int32_t *seq, int64_t idx)
{
    sol_t s;
    if (sol_alloc(&s, in->V, in->M)) return OR_ENOMEM;
    sol_from_flat(&s, off, seq);
    move_t mv;
    int ok = decode(in, &s, idx, &mv);
    if (ok) { apply_move(&s, &mv); sol_to_flat(&s, off, seq); }
    sol_free(&s);
    return ok ? OR_OK : OR_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Move keys: Algorithm 3's tabu skip and its best-candidate bookkeeping      */
/* (CurrentMin) turned into one ordered 64-bit key per slot:                  */
/*   bit 63      the move is tabu and does not beat the best objective,       */
/*   bits 62..32 delta + 2^30,                                                */
/*   bits 31..0  slot index;                                                  */
/* a slot that is not a move gets all ones.  The smallest key wins: allowed   */
/* moves first, then the smallest delta, then the smallest index.             */
/* A move is tabu if it puts a mission into a vehicle that the mission left   */
/* within the last `tenure` iterations (tabu_until[m*V + v] >= t).            */
/* ------------------------------------------------------------------------ */
static uint64_t make_key(int blocked, int64_t delta, int64_t idx)
{
    return ((uint64_t)(blocked ? 1 : 0) << 63)
         | ((uint64_t)(uint32_t)(delta + (1LL << 30)) << 32)
         | (uint64_t)(uint32_t)idx;
}

typedef struct {
    const or_inst *in;
    sol_t s;
    int32_t *route_of, *pos_of;   /* per mission */
} view_t;

static void view_index(view_t *w) { index_missions(&w->s, w->route_of, w->pos_of); }

/* Keys of every slot in index order (incremental deltas).  Calls visit(key)
 * per slot; returns the minimum. */
static uint64_t scan_keys(const or_inst *in, view_t *w, const int32_t *tabu_until,
                          int32_t t, int64_t cur, int64_t best, const or_params *pr,
                          uint64_t *keys_out)
{
    int32_t M = in->M, V = in->V;
    const sol_t *s = &w->s;
    uint64_t kmin = UINT64_MAX;
    int64_t idx = 0;
    int use_tabu = pr->variant == 0;
    /* relocates */
    for (int32_t m = 0; m < M; ++m) {
        int32_t sv = w->route_of[m], sk = w->pos_of[m];
        int32_t xP = exit_loc(in, s, sv, sk - 1), yN = enter_loc(in, s, sv, sk + 1);
        int64_t rem = (int64_t)TT(in, xP, yN) - TT(in, xP, in->p[m]) - TT(in, in->d[m], yN);
        for (int32_t v = 0; v < V; ++v) {
            int tabu = use_tabu && tabu_until[(int64_t)m * V + v] >= t;
            for (int32_t g = 0; g <= s->len[v]; ++g, ++idx) {
                uint64_t key = UINT64_MAX;
                if (!(v == sv && (g == sk || g == sk + 1))) {
                    int32_t xa = exit_loc(in, s, v, g - 1), yb = enter_loc(in, s, v, g);
                    int64_t dlt = rem + TT(in, xa, in->p[m]) + TT(in, in->d[m], yb) - TT(in, xa, yb);
                    int blocked = tabu && !(pr->aspiration && cur + dlt < best);
                    key = make_key(blocked, dlt, idx);
                }
                if (keys_out) keys_out[idx] = key;
                if (key < kmin) kmin = key;
            }
        }
    }
    /* swaps */
    move_t mv;
    memset(&mv, 0, sizeof(mv));
    mv.is_swap = 1;
    for (int32_t m1 = 0; m1 < M; ++m1) {
        for (int32_t m2 = m1 + 1; m2 < M; ++m2, ++idx) {
            mv.m1 = m1; mv.m2 = m2;
            int64_t dlt = delta_inc(in, s, w->route_of, w->pos_of, &mv);
            int tabu = use_tabu && (tabu_until[(int64_t)m1 * V + w->route_of[m2]] >= t
                                    || tabu_until[(int64_t)m2 * V + w->route_of[m1]] >= t);
            int blocked = tabu && !(pr->aspiration && cur + dlt < best);
            uint64_t key = make_key(blocked, dlt, idx);
            if (keys_out) keys_out[idx] = key;
            if (key < kmin) kmin = key;
        }
    }
    return kmin;
}

/* Public: every slot's key for a given state. */
int or_keys(const or_inst *in, const int32_t *off, const int32_t *seq,
            const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
            const or_params *pr, uint64_t *keys_out)
{
    int rc = check_inst(in);
    if (rc) return rc;
    view_t w;
    w.in = in;
    if (sol_alloc(&w.s, in->V, in->M)) return OR_ENOMEM;
    w.route_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
    w.pos_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
    sol_from_flat(&w.s, off, seq);
    view_index(&w);
    scan_keys(in, &w, tabu_until, t, cur, best, pr, keys_out);
    free(w.route_of); free(w.pos_of); sol_free(&w.s);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One iteration (Algorithm 3; Algorithm 2 when variant == 1).                */
/* State: flattened routes, tabu table, iteration t, current and best         */
/* objective.  Outputs the trace record of the iteration.                     */
/* Returns 1 if a move was applied, 0 if none (no move exists, or the         */
/* neighbourhood search found no improving move), negative on error.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t move;     /* slot index, UINT32_MAX for none */
    int32_t delta;
    int64_t obj;       /* current objective after the iteration */
    uint8_t flags;     /* bit0 swap, bit1 tabu but aspirated, bit2 all admissible moves tabu (fallback) */
} or_trace;

static int step(const or_inst *in, view_t *w, int32_t *tabu_until, int32_t t,
                int64_t *cur, int64_t *best, const or_params *pr, or_trace *tr)
{
    uint64_t kmin = scan_keys(in, w, tabu_until, t, *cur, *best, pr, NULL);
    tr->move = UINT32_MAX; tr->delta = 0; tr->obj = *cur; tr->flags = 0;
    if (kmin == UINT64_MAX) return 0;
    int blocked = (int)(kmin >> 63);
    int64_t dlt = (int64_t)((kmin >> 32) & 0x7FFFFFFFu) - (1LL << 30);
    int64_t idx = (int64_t)(kmin & 0xFFFFFFFFu);
    if (pr->variant == 1 && dlt >= 0) return 0;   /* local optimum: stop */
    move_t mv;
    decode(in, &w->s, idx, &mv);
    int32_t V = in->V;
    int was_tabu;
    if (!mv.is_swap) {
        was_tabu = tabu_until[(int64_t)mv.m * V + mv.v] >= t;
    } else {
        was_tabu = tabu_until[(int64_t)mv.m1 * V + w->route_of[mv.m2]] >= t
                || tabu_until[(int64_t)mv.m2 * V + w->route_of[mv.m1]] >= t;
    }
    if (pr->variant == 1) was_tabu = 0;
    /* tabu bookkeeping: the moved missions may not return to the vehicle they
     * leave for `tenure` iterations */
    if (pr->variant == 0) {
        if (!mv.is_swap) {
            tabu_until[(int64_t)mv.m * V + w->route_of[mv.m]] = t + pr->tenure;
        } else {
            int32_t r1 = w->route_of[mv.m1], r2 = w->route_of[mv.m2];
            tabu_until[(int64_t)mv.m1 * V + r1] = t + pr->tenure;
            tabu_until[(int64_t)mv.m2 * V + r2] = t + pr->tenure;
        }
    }
    apply_move(&w->s, &mv);
    view_index(w);
    *cur += dlt;
    tr->move = (uint32_t)idx;
    tr->delta = (int32_t)dlt;
    tr->obj = *cur;
    tr->flags = (uint8_t)((mv.is_swap ? 1 : 0) | ((was_tabu && !blocked) ? 2 : 0) | (blocked ? 4 : 0));
    if (*cur < *best) *best = *cur;
    return 1;
}

/* Public single step on flattened state (for invariant tests). */
int or_step(const or_inst *in, int32_t *off, int32_t *seq, int32_t *tabu_until,
            int32_t t, int64_t *cur, int64_t *best, const or_params *pr,
            uint32_t *tr_move, int32_t *tr_delta, int64_t *tr_obj, uint8_t *tr_flags)
{
    int rc = check_inst(in);
    if (rc) return rc;
    view_t w;
    w.in = in;
    if (sol_alloc(&w.s, in->V, in->M)) return OR_ENOMEM;
    w.route_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
    w.pos_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->M + 1));
    sol_from_flat(&w.s, off, seq);
    view_index(&w);
    or_trace tr;
    int applied = step(in, &w, tabu_until, t, cur, best, pr, &tr);
    sol_to_flat(&w.s, off, seq);
    *tr_move = tr.move; *tr_delta = tr.delta; *tr_obj = tr.obj; *tr_flags = tr.flags;
    free(w.route_of); free(w.pos_of); sol_free(&w.s);
    return applied;
}

/* ------------------------------------------------------------------------ */
/* Public: whole search.                                                      */
/*   Tabu search runs exactly max_iters iterations (an iteration with no      */
/*   move at all records UINT32_MAX); the neighbourhood search stops at the   */
/*   first iteration without an improving move, or at max_iters.            */
/*   best_*: the best solution seen (the greedy start counts, best_iter = -1) */
/*   final_*: the solution after the last iteration.                          */
/*   Trace arrays may be NULL; otherwise they hold iters_done records.        */
/* ------------------------------------------------------------------------ */
int or_solve(const or_inst *in, const or_params *pr,
             int32_t *best_off, int32_t *best_seq, int32_t *final_off, int32_t *final_seq,
             int64_t *best_obj, int64_t *final_obj, int32_t *iters_done, int32_t *best_iter,
             uint32_t *tr_move, int32_t *tr_delta, int64_t *tr_obj, uint8_t *tr_flags)
{
    int rc = check_inst(in);
    if (rc) return rc;
    if (pr->tenure < 0 || pr->max_iters < 0 || (pr->variant != 0 && pr->variant != 1)) return OR_EINVAL;
    int32_t M = in->M, V = in->V;
    view_t w;
    w.in = in;
    if (sol_alloc(&w.s, V, M)) return OR_ENOMEM;
    w.route_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    w.pos_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t *tabu = (int32_t *)malloc(sizeof(int32_t) * (size_t)M * (size_t)V + 4);
    for (int64_t k = 0; k < (int64_t)M * V; ++k) tabu[k] = -1;
    greedy(in, pr->restart_seed, &w.s);
    view_index(&w);
    int64_t cur = sol_objective(in, &w.s), best = cur;
    int32_t bi = -1, done = 0;
    sol_to_flat(&w.s, best_off, best_seq);
    for (int32_t t = 0; t < pr->max_iters; ++t) {
        or_trace tr;
        int64_t prev_best = best;
        int applied = step(in, &w, tabu, t, &cur, &best, pr, &tr);
        if (pr->variant == 1 && !applied) break;
        if (tr_move) { tr_move[t] = tr.move; tr_delta[t] = tr.delta; tr_obj[t] = tr.obj; tr_flags[t] = tr.flags; }
        done = t + 1;
        if (best < prev_best) { bi = t; sol_to_flat(&w.s, best_off, best_seq); }
    }
    sol_to_flat(&w.s, final_off, final_seq);
    *best_obj = best; *final_obj = cur; *iters_done = done; *best_iter = bi;
    free(tabu); free(w.route_of); free(w.pos_of); sol_free(&w.s);
    return OR_OK;
}

int64_t or_num_slots(int32_t M, int32_t V) { return n_slots(M, V); }
