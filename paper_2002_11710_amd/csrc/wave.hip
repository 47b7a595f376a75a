// wave.hip -- one wavefront per solve, the whole state in LDS.
//
// The schedule for small solves (a wavefront holds a solve: no workgroup
// barriers, several solves per workgroup), for the constrained model of
// Section 3 (two vehicle types with their own travel matrices, time limits at
// the delivery points with waiting, a horizon, a flight limit, helicopter-only
// missions: Eqs (7)-(10)) and for the sweep form of Algorithms 2 and 3.
//
// A solve's LDS region holds the compact travel block of each vehicle type
// (exit rows x entry columns, staged from the caller's matrices with the
// numbering the prepare kernel made), per-mission and per-vehicle constants,
// the routes (flat array, offsets, vehicle of each position, position and
// vehicle of each mission), the tabu table [vehicle][mission] and the records
// each iteration rebuilds:
//   per mission m (its neighbours P before and N after it in its route):
//     mx   exit row of P,  my  entry column of N,
//     mlv  time the vehicle leaves P (0 at the base, else P's time limit),
//     mlat latest arrival at N's pickup (N's limit minus its loaded leg, or the
//          horizon for the base),
//     mout t(P->m) + t(m->N) + loaded leg of m, mrem t(P->N) - mout,
//     mok  the flight P->N is feasible (m may leave its route);
//   per gap G (between A and B in vehicle gv's route): gx exit row of A, gy
//     entry column of B, glv time leaving A, glat latest arrival at B, gc t(A->B).
// Every time is in the matrix of the route's vehicle type.  Because a vehicle
// always leaves a mission at its time limit, whether a flight x -> y is
// feasible depends on x and y alone, so a move is feasible exactly when the
// flights it creates are, its missions are compatible with their new vehicles
// and the routes it changes stay within the flight limit.
//
// Best form, per iteration: records -> every slot's key (the 64-bit key of the
// other schedules: blocked << 63 | (delta + 2^30) << 32 | slot index, with a
// move that breaks a constraint scored as no move) in slot order over the
// lanes -> wavefront minimum -> decode and apply.  Sweep form: per mission
// turn, that mission's relocates to other vehicles only, strictly improving.
#include "atabu_internal.h"
#include "atabu.h"

namespace at {

namespace {

constexpr uint64_t kG = 0x9E3779B97F4A7C15ull;
constexpr int32_t kBig = 0x3FFFFFFF;   // an unreachable time (no limit)

__device__ __forceinline__ uint64_t wmin(uint64_t k) { return wave_min_u64(k); }

// all lanes' LDS writes before this point are seen by all lanes' reads after it
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the k-th output (k >= 1) of SplitMix64(seed)
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * kG;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t key_of(bool blocked, int d, uint32_t idx)
{
    return ((uint64_t)blocked << 63) | ((uint64_t)(uint32_t)(d + kDeltaBias) << 32) | idx;
}

struct WLay {
    uint32_t tc0, tc1, mrow, mcol, vrow, vcol, svc0, svc1, w, heli, vtype, cost;
    uint32_t seq, off, rt, pof, rof, tabu;
    uint32_t gx, gy, gv, glv, glat, gc;
    uint32_t mx, my, mlv, mlat, mout, mrem, mok;
    uint32_t ord, aux, red, total;
};

__host__ __device__ inline uint32_t a16(uint64_t x) { return (uint32_t)((x + 15u) & ~15ull); }

__host__ __device__ inline WLay wave_layout(int M, int V, int R, int Cs, int esz, bool two)
{
    WLay l;
    uint64_t o = 0;
    const uint64_t uM = (uint64_t)M, uV = (uint64_t)V, NG = uM + uV;
#define W_TAKE(f, bytes) do { l.f = (uint32_t)o; o = a16(o + (uint64_t)(bytes)); } while (0)
    W_TAKE(tc0, (uint64_t)R * Cs * esz);
    W_TAKE(tc1, two ? (uint64_t)R * Cs * esz : 0);
    W_TAKE(mrow, 4 * uM); W_TAKE(mcol, 4 * uM); W_TAKE(vrow, 4 * uV); W_TAKE(vcol, 4 * uV);
    W_TAKE(svc0, 4 * uM); W_TAKE(svc1, two ? 4 * uM : 0);
    W_TAKE(w, 4 * uM); W_TAKE(heli, 4 * uM); W_TAKE(vtype, 4 * uV); W_TAKE(cost, 4 * uV);
    W_TAKE(seq, 4 * uM); W_TAKE(off, 4 * (uV + 1)); W_TAKE(rt, 4 * uM); W_TAKE(pof, 4 * uM);
    W_TAKE(rof, 4 * uM); W_TAKE(tabu, 4 * uM * uV);
    W_TAKE(gx, 4 * NG); W_TAKE(gy, 4 * NG); W_TAKE(gv, 4 * NG); W_TAKE(glv, 4 * NG);
    W_TAKE(glat, 4 * NG); W_TAKE(gc, 4 * NG);
    W_TAKE(mx, 4 * uM); W_TAKE(my, 4 * uM); W_TAKE(mlv, 4 * uM); W_TAKE(mlat, 4 * uM);
    W_TAKE(mout, 4 * uM); W_TAKE(mrem, 4 * uM); W_TAKE(mok, 4 * uM);
    W_TAKE(ord, 4 * NG); W_TAKE(aux, 4 * NG); W_TAKE(red, 64);
#undef W_TAKE
    l.total = o > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)o;
    return l;
}

template <typename TE>
struct W {
    // the two vehicle types' travel blocks and loaded legs: picked by a select,
    // never by an index, so the struct stays in registers
    TE *tc0, *tc1;
    int32_t *svc0, *svc1;
    int32_t *mrow, *mcol, *vrow, *vcol, *w, *heli, *vtype, *cost;
    int32_t *seq, *off, *rt, *pof, *rof, *tabu;
    int32_t *gx, *gy, *gv, *glv, *glat, *gc;
    int32_t *mx, *my, *mlv, *mlat, *mout, *mrem, *mok;
    int32_t *ord, *aux;
    int64_t *red;
    int M, V, H, FL;
    bool useW, useH, useFL;   // time limits, helicopter-only missions, flight limit

    __device__ TE *tcp(int ty) const { return ty ? tc1 : tc0; }
    __device__ int32_t *svcp(int ty) const { return ty ? svc1 : svc0; }
    __device__ int tv(int v, int x) const { return (int)tcp(vtype[v])[x]; }
};

template <typename TE>
__device__ W<TE> make_w(char *base, const WLay &l, const InstDev &I)
{
    W<TE> c;
    const bool two = I.T2 != nullptr;
    c.tc0 = (TE *)(base + l.tc0);
    c.tc1 = two ? (TE *)(base + l.tc1) : c.tc0;
    c.mrow = (int32_t *)(base + l.mrow); c.mcol = (int32_t *)(base + l.mcol);
    c.vrow = (int32_t *)(base + l.vrow); c.vcol = (int32_t *)(base + l.vcol);
    c.svc0 = (int32_t *)(base + l.svc0);
    c.svc1 = two ? (int32_t *)(base + l.svc1) : c.svc0;
    c.w = (int32_t *)(base + l.w); c.heli = (int32_t *)(base + l.heli);
    c.vtype = (int32_t *)(base + l.vtype); c.cost = (int32_t *)(base + l.cost);
    c.seq = (int32_t *)(base + l.seq); c.off = (int32_t *)(base + l.off);
    c.rt = (int32_t *)(base + l.rt); c.pof = (int32_t *)(base + l.pof);
    c.rof = (int32_t *)(base + l.rof); c.tabu = (int32_t *)(base + l.tabu);
    c.gx = (int32_t *)(base + l.gx); c.gy = (int32_t *)(base + l.gy); c.gv = (int32_t *)(base + l.gv);
    c.glv = (int32_t *)(base + l.glv); c.glat = (int32_t *)(base + l.glat); c.gc = (int32_t *)(base + l.gc);
    c.mx = (int32_t *)(base + l.mx); c.my = (int32_t *)(base + l.my); c.mlv = (int32_t *)(base + l.mlv);
    c.mlat = (int32_t *)(base + l.mlat); c.mout = (int32_t *)(base + l.mout);
    c.mrem = (int32_t *)(base + l.mrem); c.mok = (int32_t *)(base + l.mok);
    c.ord = (int32_t *)(base + l.ord); c.aux = (int32_t *)(base + l.aux);
    c.red = (int64_t *)(base + l.red);
    c.M = uniform(I.M); c.V = uniform(I.V);
    c.useW = I.w != nullptr;
    c.useH = I.heli != nullptr;
    c.useFL = uniform(I.flimit) > 0;
    c.H = c.useW ? uniform(I.horizon) : kBig;
    c.FL = c.useFL ? uniform(I.flimit) : 0x7FFFFFFF;
    return c;
}

// Stage the instance into LDS.  Returns a status (AT_OK, or AT_ERANGE /
// AT_EINVAL for constrained-model inputs out of range), uniform over the wave.
template <typename TE>
__device__ int stage(const InstDev &I, const W<TE> &c, int lane)
{
    const int L = uniform(I.L), R = uniform(I.R), C = uniform(I.C), Cs = uniform(I.Cs);
    const int M = uniform(I.M), V = uniform(I.V);
    int bad = AT_OK;
    const int32_t *Ts[2] = {I.T, I.T2 ? I.T2 : I.T};
    const int nt = I.T2 ? 2 : 1;
    for (int k = 0; k < nt; ++k)
        for (int e = lane; e < R * Cs; e += kWave) {
            const int r = e / Cs, col = e - r * Cs;
            int x = 0;
            if (col < C) x = Ts[k][(int64_t)I.exit_loc[r] * L + I.enter_loc[col]];
            if (x < 0 || x >= kMaxTravel) bad = AT_ERANGE;
            c.tcp(k)[e] = (TE)x;
        }
    for (int m = lane; m < M; m += kWave) {
        c.mrow[m] = I.mrow[m];
        c.mcol[m] = I.mcol[m];
        const int64_t pd = (int64_t)I.p[m] * L + I.d[m];
        c.svc0[m] = I.T[pd];
        if (I.T2) {
            const int x = I.T2[pd];
            if (x < 0 || x >= kMaxTravel) bad = AT_ERANGE;
            c.svc1[m] = x;
        }
        const int wm = I.w ? I.w[m] : 0;
        const int hm = I.heli ? I.heli[m] : 0;
        if (wm < 0 || wm > kBig - kMaxTravel * 4 || hm < 0 || hm > 1) bad = AT_EINVAL;
        c.w[m] = wm;
        c.heli[m] = hm;
    }
    for (int v = lane; v < V; v += kWave) {
        c.vrow[v] = I.vrow[v];
        c.vcol[v] = I.vcol[v];
        const int ty = I.vtype ? I.vtype[v] : 0;
        if (ty < 0 || ty > 1 || (ty == 1 && !I.T2)) bad = AT_EINVAL;
        c.vtype[v] = ty > 0 ? 1 : 0;
    }
    // the first error of any lane, uniform over the wave
    int e = bad;
    for (int o = 32; o > 0; o >>= 1) { const int x = __shfl_xor(e, o, 64); e = x < e ? x : e; }
    wsync();
    return e;
}

// Records of the current routes (the first Mp positions hold the placed
// missions; Mp < M only inside the greedy start).
template <typename TE>
__device__ void prep(const W<TE> &c, int Mp, int lane)
{
    for (int i = lane; i < Mp; i += kWave) {
        const int m = c.seq[i], r = c.rt[i], ty = c.vtype[r];
        const TE *tc = c.tcp(ty);
        const int32_t *svc = c.svcp(ty);
        const bool first = i == c.off[r], last = i + 1 == c.off[r + 1];
        const int pm = first ? -1 : c.seq[i - 1], nm = last ? -1 : c.seq[i + 1];
        const int x = first ? c.vrow[r] : c.mrow[pm];
        const int y = last ? c.vcol[r] : c.mcol[nm];
        const int lv = (first || !c.useW) ? 0 : c.w[pm];
        const int lat = last ? c.H : (c.useW ? c.w[nm] - svc[nm] : kBig);
        const int tPX = (int)tc[x + c.mcol[m]], tXN = (int)tc[c.mrow[m] + y], tPN = (int)tc[x + y];
        const int out = tPX + tXN + svc[m];
        c.mx[m] = x; c.my[m] = y; c.mlv[m] = lv; c.mlat[m] = lat;
        c.mout[m] = out; c.mrem[m] = tPN - out;
        c.mok[m] = (!c.useW || lv + tPN <= lat) ? 1 : 0;
        const int G = i + r;   // the gap before position i: A = P, B = m
        c.gx[G] = x; c.gy[G] = c.mcol[m]; c.gv[G] = r; c.glv[G] = lv;
        c.glat[G] = c.useW ? c.w[m] - svc[m] : kBig;
        c.gc[G] = tPX;
    }
    for (int r = lane; r < c.V; r += kWave) {
        const int e = c.off[r + 1], ty = c.vtype[r];
        const bool empty = c.off[r] == e;
        const int lm = empty ? -1 : c.seq[e - 1];
        const int x = empty ? c.vrow[r] : c.mrow[lm];
        const int G = e + r;   // the gap before the return to base
        c.gx[G] = x; c.gy[G] = c.vcol[r]; c.gv[G] = r;
        c.glv[G] = (empty || !c.useW) ? 0 : c.w[lm];
        c.glat[G] = c.H;
        c.gc[G] = (int)c.tcp(ty)[x + c.vcol[r]];
        if (c.useFL) {
            // the route's flight time in its own matrix
            int s = 0, prevx = c.vrow[r];
            for (int k = c.off[r]; k < e; ++k) {
                const int m = c.seq[k];
                s += (int)c.tcp(ty)[prevx + c.mcol[m]] + c.svcp(ty)[m];
                prevx = c.mrow[m];
            }
            if (!empty) s += (int)c.tcp(ty)[prevx + c.vcol[r]];
            c.cost[r] = s;
        }
    }
    wsync();
}

// Delta and feasibility of relocating mission m into gap G.  The conditions are
// combined without branches, so the loads of consecutive slots can overlap.
template <typename TE>
__device__ __forceinline__ bool relocate_eval(const W<TE> &c, int m, int G, int &d)
{
    const int v = c.gv[G], ty = c.vtype[v], src = c.rof[m];
    const TE *tc = c.tcp(ty);
    const int sv = c.svcp(ty)[m];
    const int tAX = (int)tc[c.gx[G] + c.mcol[m]], tXB = (int)tc[c.mrow[m] + c.gy[G]];
    const int ins = tAX + tXB - c.gc[G] + sv;
    d = c.mrem[m] + ins;
    bool ok = true;
    if (c.useH) ok &= !(c.heli[m] != 0 && ty == 1);
    if (c.useW) {
        const int wm = c.w[m];
        ok &= (c.mok[m] != 0) & (c.glv[G] + tAX + sv <= wm) & (wm + tXB <= c.glat[G]);
    }
    if (c.useFL) {
        const int cv = c.cost[v], cs = c.cost[src];
        ok &= v == src ? cv + d <= c.FL : (cs + c.mrem[m] <= c.FL) & (cv + ins <= c.FL);
    }
    return ok;
}

// Delta and feasibility of swapping missions a and b.
template <typename TE>
__device__ __forceinline__ bool swap_eval(const W<TE> &c, int a, int b, int &d)
{
    const int pa = c.pof[a], pb = c.pof[b], ra = c.rof[a], rb = c.rof[b];
    if (ra == rb && (pb == pa + 1 || pa == pb + 1)) {
        const int F = pa < pb ? a : b, S = pa < pb ? b : a;
        const int ty = c.vtype[ra];
        const TE *tc = c.tcp(ty);
        const int32_t *svc = c.svcp(ty);
        const int tPS = (int)tc[c.mx[F] + c.mcol[S]], tSF = (int)tc[c.mrow[S] + c.mcol[F]];
        const int tFN = (int)tc[c.mrow[F] + c.my[S]], tFS = (int)tc[c.mrow[F] + c.mcol[S]];
        d = tPS + tSF + tFN + svc[S] + svc[F] - (c.mout[F] + c.mout[S] - tFS);
        if (c.useW && (c.mlv[F] + tPS + svc[S] > c.w[S] || c.w[S] + tSF + svc[F] > c.w[F] ||
                       c.w[F] + tFN > c.mlat[S]))
            return false;
        if (c.useFL && c.cost[ra] + d > c.FL) return false;
        return true;
    }
    const int ta = c.vtype[ra], tb = c.vtype[rb];
    const TE *tca = c.tcp(ta), *tcb = c.tcp(tb);
    const int tPb = (int)tca[c.mx[a] + c.mcol[b]], tbN = (int)tca[c.mrow[b] + c.my[a]];
    const int tPa = (int)tcb[c.mx[b] + c.mcol[a]], taN = (int)tcb[c.mrow[a] + c.my[b]];
    const int sb = c.svcp(ta)[b], sa = c.svcp(tb)[a];
    const int da = tPb + tbN + sb - c.mout[a], db = tPa + taN + sa - c.mout[b];
    d = da + db;
    if (c.useH && ((c.heli[b] && ta == 1) || (c.heli[a] && tb == 1))) return false;
    if (c.useW && (c.mlv[a] + tPb + sb > c.w[b] || c.w[b] + tbN > c.mlat[a] ||
                   c.mlv[b] + tPa + sa > c.w[a] || c.w[a] + taN > c.mlat[b]))
        return false;
    if (c.useFL) {
        if (ra == rb) {
            if (c.cost[ra] + d > c.FL) return false;
        } else if (c.cost[ra] + da > c.FL || c.cost[rb] + db > c.FL) {
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ uint32_t swap_idx(uint32_t R, uint32_t M, uint32_t a, uint32_t b)
{
    return R + a * M - (a * (a + 1u)) / 2u + (b - a - 1u);
}

// This lane's minimum key over every slot (best form); with `keys`, every
// slot's key is also written out (the key dump).
template <typename TE>
__device__ uint64_t eval_best(const W<TE> &c, int lane, int t, int thr, bool use_tabu, uint64_t *keys)
{
    const int M = c.M, V = c.V, NG = M + V;
    const uint32_t R = (uint32_t)M * (uint32_t)NG;
    uint64_t best = kKeyNone;
    // relocates: slot m*NG + G, lanes over consecutive slots, two slots of a lane
    // per step (their loads in flight together)
    int m = 0, G = lane;
    while (G >= NG && m < M) { G -= NG; ++m; }
    auto reloc_key = [&](int mm, int GG) {
        const int s = c.pof[mm] + c.rof[mm];
        int d;
        const bool ok = relocate_eval(c, mm, GG, d);
        const bool tb = use_tabu && c.tabu[c.gv[GG] * M + mm] > t;
        return ((unsigned)(GG - s) >= 2u && ok) ? key_of(tb && !(d < thr), d, (uint32_t)mm * (uint32_t)NG + (uint32_t)GG)
                                                 : kKeyNone;
    };
    while (m < M) {
        const int m1 = m, G1 = G;
        G += kWave;
        while (G >= NG && m < M) { G -= NG; ++m; }
        const bool two = m < M;
        const int m2 = two ? m : m1, G2 = two ? G : G1;
        const uint64_t k1 = reloc_key(m1, G1), k2 = reloc_key(m2, G2);
        if (keys) {
            keys[(uint32_t)m1 * (uint32_t)NG + (uint32_t)G1] = k1;
            if (two) keys[(uint32_t)m2 * (uint32_t)NG + (uint32_t)G2] = k2;
        }
        best = k1 < best ? k1 : best;
        best = (two && k2 < best) ? k2 : best;
        if (two) {
            G += kWave;
            while (G >= NG && m < M) { G -= NG; ++m; }
        }
    }
    // swaps: slot R + a*M - a(a+1)/2 + (b-a-1), lanes over consecutive slots
    const int64_t nsw = (int64_t)M * (M - 1) / 2;
    if (nsw > 0) {
        int a = 0, b = 1 + lane;
        while (a < M - 1 && b >= M) { b -= M - a - 1; ++a; b += 1; }
        for (int64_t sidx = lane; sidx < nsw; sidx += kWave) {
            int d;
            uint64_t k = kKeyNone;
            const uint32_t idx = swap_idx(R, (uint32_t)M, (uint32_t)a, (uint32_t)b);
            if (swap_eval(c, a, b, d)) {
                const bool tb = use_tabu && (c.tabu[c.rof[b] * M + a] > t || c.tabu[c.rof[a] * M + b] > t);
                k = key_of(tb && !(d < thr), d, idx);
            }
            if (keys) keys[idx] = k;
            best = k < best ? k : best;
            b += kWave;
            while (a < M - 1 && b >= M) { b -= M - a - 1; ++a; b += 1; }
        }
    }
    return best;
}

// Move mission m (placed at position s on vehicle rs) to flat position q on
// vehicle v; the positions between shift by one, 64 at a time, each chunk read
// into registers before it is written, chunks taken in the direction of the
// shift.  With s = Mp (not placed) it is an insertion at q.
template <typename TE>
__device__ void move_to(const W<TE> &c, int m, int s, int rs, int q, int v, int lane)
{
    if (q > s) {
        for (int c0 = s; c0 < q; c0 += kWave) {
            const int k = c0 + lane;
            int sm = 0, sr = 0;
            if (k < q) { sm = c.seq[k + 1]; sr = c.rt[k + 1]; }
            wsync();
            if (k < q) { c.seq[k] = sm; c.rt[k] = sr; c.pof[sm] = k; }
            wsync();
        }
    } else if (q < s) {
        for (int c0 = s; c0 > q; c0 -= kWave) {
            const int k = c0 - lane;
            int sm = 0, sr = 0;
            if (k > q) { sm = c.seq[k - 1]; sr = c.rt[k - 1]; }
            wsync();
            if (k > q) { c.seq[k] = sm; c.rt[k] = sr; c.pof[sm] = k; }
            wsync();
        }
    }
    if (lane == 0) { c.seq[q] = m; c.rt[q] = v; c.pof[m] = q; c.rof[m] = v; }
    if (rs < 0) {
        for (int r = v + 1 + lane; r <= c.V; r += kWave) c.off[r] += 1;
    } else if (v > rs) {
        for (int r = rs + 1 + lane; r <= v; r += kWave) c.off[r] -= 1;
    } else if (v < rs) {
        for (int r = v + 1 + lane; r <= rs; r += kWave) c.off[r] += 1;
    }
    wsync();
}

// Apply relocate (m, G) to the routes (gap numbering before the move).
template <typename TE>
__device__ void apply_relocate(const W<TE> &c, int m, int G, int lane)
{
    const int v = c.gv[G], s = c.pof[m], rs = c.rof[m];
    const int fp = G - v;
    const int q = fp - (fp > s ? 1 : 0);
    wsync();
    move_to(c, m, s, rs, q, v, lane);
}

template <typename TE>
__device__ void apply_swap(const W<TE> &c, int a, int b, int lane)
{
    const int pa = c.pof[a], pb = c.pof[b], ra = c.rof[a], rb = c.rof[b];
    wsync();
    if (lane == 0) {
        c.seq[pa] = b; c.seq[pb] = a;
        c.pof[a] = pb; c.pof[b] = pa;
        c.rof[a] = rb; c.rof[b] = ra;
    }
    wsync();
}

// One mission's turn of the sweep form: the smallest negative-delta relocate
// of j to a gap of another vehicle (ties: smallest gap), compatible, feasible
// and, with tabu on, not to a listed vehicle.  Returns its key
// ((delta + 2^30) << 32 | G) or kKeyNone.
template <typename TE>
__device__ uint64_t sweep_choice(const W<TE> &c, int j, int Mp, int turn, bool use_tabu, int lane)
{
    const int NG = Mp + c.V, own = c.rof[j];
    uint64_t best = kKeyNone;
    for (int G = lane; G < NG; G += kWave) {
        const int v = c.gv[G];
        if (v == own) continue;
        if (use_tabu && c.tabu[v * c.M + j] > turn) continue;
        int d;
        if (relocate_eval(c, j, G, d) && d < 0) {
            const uint64_t k = ((uint64_t)(uint32_t)(d + kDeltaBias) << 32) | (uint32_t)G;
            best = k < best ? k : best;
        }
    }
    return wmin(best);
}

// One pass of the sweep form.  Vehicles in order (Fisher-Yates from the draw
// stream when seed != 0), each vehicle's missions as they stand when its turn
// begins (likewise shuffled).  *nd counts the draws taken; *turn the turns;
// per turn the trace record when tr_move is set.  Returns the missions moved
// (-1 if the turn budget ran out first).
template <typename TE>
__device__ int sweep_pass(const W<TE> &c, const JobDev &J, int Mp, bool use_tabu, int tenure,
                          uint64_t seed, uint64_t *nd, int *turn, int max_turns, int64_t *cur,
                          int *last_move, bool trace, int lane)
{
    const int V = c.V;
    int moved = 0;
    int32_t *vord = c.aux + Mp;    // V entries after the mission list
    if (lane == 0) {
        for (int v = 0; v < V; ++v) vord[v] = v;
        if (seed)
            for (int i = V - 1; i >= 1; --i) {
                const int j = (int)(draw(seed, ++*nd) % (uint64_t)(i + 1));
                const int x = vord[i]; vord[i] = vord[j]; vord[j] = x;
            }
    }
    *nd = (uint64_t)__shfl((long long)*nd, 0, 64);
    wsync();
    for (int vi = 0; vi < V; ++vi) {
        const int i = vord[vi];
        const int o0 = c.off[i], n = c.off[i + 1] - o0;
        for (int k = lane; k < n; k += kWave) c.aux[k] = c.seq[o0 + k];
        wsync();
        if (seed && lane == 0)
            for (int q = n - 1; q >= 1; --q) {
                const int j = (int)(draw(seed, ++*nd) % (uint64_t)(q + 1));
                const int x = c.aux[q]; c.aux[q] = c.aux[j]; c.aux[j] = x;
            }
        *nd = (uint64_t)__shfl((long long)*nd, 0, 64);
        wsync();
        for (int q = 0; q < n; ++q) {
            if (*turn >= max_turns) return -1;
            const int j = c.aux[q];
            prep(c, Mp, lane);
            const uint64_t k = sweep_choice(c, j, Mp, *turn, use_tabu, lane);
            uint32_t rec = 0xFFFFFFFFu;
            int d = 0;
            if (k != kKeyNone) {
                d = (int)(uint32_t)(k >> 32) - kDeltaBias;
                const int G = (int)(uint32_t)k;
                const int left = c.rof[j];
                rec = (uint32_t)j * (uint32_t)(c.M + V) + (uint32_t)G;
                apply_relocate(c, j, G, lane);
                if (use_tabu && lane == 0) c.tabu[left * c.M + j] = *turn + tenure;
                *cur += d;
                *last_move = *turn;
                ++moved;
            }
            if (trace && lane == 0) {
                J.tr_move[*turn] = rec;
                J.tr_delta[*turn] = d;
                J.tr_obj[*turn] = *cur;
                J.tr_flags[*turn] = 0;
            }
            ++*turn;
            wsync();
        }
    }
    return moved;
}

// Objective of the current routes (every vehicle in its own matrix).
template <typename TE>
__device__ int64_t objective(const W<TE> &c, int lane)
{
    int64_t s = 0;
    for (int r = lane; r < c.V; r += kWave) {
        const int ty = c.vtype[r], e = c.off[r + 1];
        if (c.off[r] == e) continue;
        int prevx = c.vrow[r];
        for (int k = c.off[r]; k < e; ++k) {
            const int m = c.seq[k];
            s += (int64_t)c.tcp(ty)[prevx + c.mcol[m]] + c.svcp(ty)[m];
            prevx = c.mrow[m];
        }
        s += (int64_t)c.tcp(ty)[prevx + c.vcol[r]];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor((long long)s, o, 64);
    return s;
}

// Algorithm 1.  Order: with the constrained model, helicopter-only missions
// first, then by time limit, then by rank in the Fisher-Yates order of
// SplitMix64(seed) (identity for seed 0); without it, that order alone.  Each
// mission is appended to the vehicle with the least added flight time among
// those where it fits (ties: lowest vehicle); where it fits nowhere, one
// neighbourhood-search sweep over the missions placed so far and one more try.
// Returns AT_OK or AT_EINFEAS.
template <typename TE>
__device__ int greedy(const W<TE> &c, uint64_t seed, int lane)
{
    const int M = c.M, V = c.V;
    // pi (the seeded order) in ord, each mission's rank in it in aux, then the
    // final order in ord (aux is the sweep's scratch, ord stays untouched)
    int32_t *pi = c.ord, *rank = c.aux, *order = c.ord;
    for (int i = lane; i < M; i += kWave) pi[i] = i;
    for (int v = lane; v <= V; v += kWave) c.off[v] = 0;
    wsync();
    if (seed != 0 && lane == 0)
        for (int i = M - 1; i >= 1; --i) {
            const int j = (int)(draw(seed, (uint64_t)(M - i)) % (uint64_t)(i + 1));
            const int x = pi[i]; pi[i] = pi[j]; pi[j] = x;
        }
    wsync();
    for (int i = lane; i < M; i += kWave) rank[pi[i]] = i;
    wsync();
    // position of each mission in the order: count the missions before it
    for (int m = lane; m < M; m += kWave) {
        const int hm = c.useH ? c.heli[m] : 0, wm = c.useW ? c.w[m] : 0, rm = rank[m];
        int pos = 0;
        for (int x = 0; x < M; ++x) {
            const int hx = c.useH ? c.heli[x] : 0, wx = c.useW ? c.w[x] : 0, rx = rank[x];
            pos += (hx != hm) ? (hx > hm) : (wx != wm) ? (wx < wm) : (rx < rm);
        }
        order[pos] = m;
    }
    for (int v = lane; v < V; v += kWave) c.cost[v] = 0;
    wsync();
    int status = AT_OK;
    for (int q = 0; q < M && status == AT_OK; ++q) {
        const int m = order[q];
        for (int attempt = 0; attempt < 2; ++attempt) {
            uint64_t k = kKeyNone;
            for (int v = lane; v < V; v += kWave) {
                const int ty = c.vtype[v];
                if (c.useH && c.heli[m] && ty == 1) continue;
                const TE *tc = c.tcp(ty);
                const int e = c.off[v + 1];
                const bool empty = c.off[v] == e;
                const int lm = empty ? -1 : c.seq[e - 1];
                const int x = empty ? c.vrow[v] : c.mrow[lm];
                const int lv = (empty || !c.useW) ? 0 : c.w[lm];
                const int sv = c.svcp(ty)[m];
                const int tLX = (int)tc[x + c.mcol[m]], tXB = (int)tc[c.mrow[m] + c.vcol[v]];
                const int add = tLX + sv + tXB - (int)tc[x + c.vcol[v]];
                if (c.useW && (lv + tLX + sv > c.w[m] || c.w[m] + tXB > c.H)) continue;
                if (c.useFL && c.cost[v] + add > c.FL) continue;
                const uint64_t kk = ((uint64_t)(uint32_t)(add + kDeltaBias) << 32) | (uint32_t)v;
                k = kk < k ? kk : k;
            }
            k = wmin(k);
            if (k != kKeyNone) {
                const int v = (int)(uint32_t)k;
                const int add = (int)(uint32_t)(k >> 32) - kDeltaBias;
                const int Mp = c.off[V];
                move_to(c, m, Mp, -1, c.off[v + 1], v, lane);
                if (lane == 0) c.cost[v] += add;
                wsync();
                break;
            }
            if (attempt == 1 || q == 0) { status = AT_EINFEAS; break; }
            // repair: one neighbourhood-search sweep over the placed missions
            const int Mp = c.off[V];
            uint64_t nd = 0;
            int turn = 0, last = -1;
            int64_t cur = 0;
            sweep_pass(c, JobDev{}, Mp, false, 0, 0, &nd, &turn, 0x7FFFFFFF, &cur, &last, false, lane);
            // the route costs after the repair
            prep(c, Mp, lane);
        }
    }
    wsync();
    return status;
}

template <typename TE>
__device__ void write_routes(const W<TE> &c, int32_t *off, int32_t *seq, int32_t *of, int lane)
{
    for (int i = lane; i < c.M; i += kWave) {
        seq[i] = c.seq[i];
        if (of) of[c.seq[i]] = c.rt[i];
    }
    for (int v = lane; v <= c.V; v += kWave) off[v] = c.off[v];
}

// Decode a best-form slot index into a move and apply it; sets the tabu
// entries (Tabu) and returns whether it was tabu at iteration t.
template <typename TE>
__device__ bool apply_best(const W<TE> &c, uint32_t idx, int t, int tenure, bool use_tabu, int lane)
{
    const int M = c.M, NG = M + c.V;
    const uint32_t R = (uint32_t)M * (uint32_t)NG;
    bool was = false;
    if (idx < R) {
        const int m = (int)(idx / (uint32_t)NG), G = (int)(idx - (uint32_t)m * (uint32_t)NG);
        const int v = c.gv[G], rs = c.rof[m];
        if (use_tabu) {
            was = c.tabu[v * M + m] > t;
            wsync();
            if (lane == 0) c.tabu[rs * M + m] = t + tenure + 1;
        }
        apply_relocate(c, m, G, lane);
    } else {
        int a, b;
        swap_pair(idx - R, M, a, b);
        const int ra = c.rof[a], rb = c.rof[b];
        if (use_tabu) {
            was = c.tabu[rb * M + a] > t || c.tabu[ra * M + b] > t;
            wsync();
            if (lane == 0) { c.tabu[ra * M + a] = t + tenure + 1; c.tabu[rb * M + b] = t + tenure + 1; }
        }
        apply_swap(c, a, b, lane);
    }
    return was;
}

template <typename TE>
__device__ void run_wave_job(const JobDev &J, char *base, int lane)
{
    const InstDev &I = *J.inst;
    const WLay ly = wave_layout(uniform(I.M), uniform(I.V), uniform(I.R), uniform(I.Cs), (int)sizeof(TE),
                                I.T2 != nullptr);
    const W<TE> c = make_w<TE>(base, ly, I);
    const int M = c.M, V = c.V;
    int status = stage(I, c, lane);
    for (int k = lane; k < M * V; k += kWave) c.tabu[k] = 0;
    if (status == AT_OK) status = greedy(c, J.seed, lane);
    wsync();
    int64_t cur = 0, best = 0;
    int t = J.t_begin, best_iter = -1;
    if (status == AT_OK) {
        cur = objective(c, lane);
        best = cur;
        write_routes(c, J.out_off, J.out_seq, J.out_of, lane);
        const bool use_tabu = J.variant == AT_TABU;
        if (J.form == AT_FORM_SWEEP) {
            uint64_t nd = 0;
            int turn = 0, last = -1;
            for (;;) {
                const int moved = sweep_pass(c, J, M, use_tabu, J.tenure, J.seed, &nd, &turn, J.t_end, &cur,
                                             &last, J.trace != 0, lane);
                if (moved <= 0) break;
            }
            t = turn;
            best = cur;
            best_iter = last;
            write_routes(c, J.out_off, J.out_seq, J.out_of, lane);
        } else {
            for (; t < J.t_end; ++t) {
                prep(c, M, lane);
                int thr = INT32_MIN;
                if (J.aspiration) {
                    const int64_t g = best - cur;
                    thr = g < (int64_t)INT32_MIN ? INT32_MIN : (int)g;
                }
                const uint64_t k = wmin(eval_best(c, lane, t, thr, use_tabu, nullptr));
                if (k == kKeyNone) {
                    if (!use_tabu) break;
                    if (J.trace && lane == 0) {
                        J.tr_move[t] = 0xFFFFFFFFu; J.tr_delta[t] = 0; J.tr_obj[t] = cur; J.tr_flags[t] = 0;
                    }
                    continue;
                }
                const bool blocked = (k >> 63) != 0;
                const int d = (int)((uint32_t)(k >> 32) & 0x7FFFFFFFu) - kDeltaBias;
                const uint32_t idx = (uint32_t)k;
                if (!use_tabu && d >= 0) break;
                const bool was = apply_best(c, idx, t, J.tenure, use_tabu, lane);
                cur += d;
                if (J.trace && lane == 0) {
                    J.tr_move[t] = idx;
                    J.tr_delta[t] = d;
                    J.tr_obj[t] = cur;
                    J.tr_flags[t] = (uint8_t)((idx >= (uint32_t)M * (uint32_t)(M + V) ? 1 : 0) |
                                              ((was && !blocked) ? 2 : 0) | (blocked ? 4 : 0));
                }
                if (cur < best) {
                    best = cur;
                    best_iter = t;
                    write_routes(c, J.out_off, J.out_seq, J.out_of, lane);
                }
            }
        }
        if (J.fin_off) write_routes(c, J.fin_off, J.fin_seq, nullptr, lane);
    }
    if (lane == 0) {
        J.scal->best_obj = best;
        J.scal->final_obj = cur;
        J.scal->iters_done = status == AT_OK ? t : 0;
        J.scal->best_iter = best_iter;
        J.scal->stopped = 0;
        J.scal->status = status;
    }
}

}  // namespace

uint32_t wave_lds_bytes(int M, int V, int R, int Cs, int esz, bool two)
{
    return wave_layout(M, V, R, Cs, esz, two).total;
}

// Each wavefront takes solves from the queue until it is empty; its LDS
// region is lds_per_solve bytes at its index within the workgroup.
template <typename TE>
__global__ void __launch_bounds__(256) k_search_wave(const JobDev *jobs, int n_jobs, uint32_t *queue,
                                                    uint32_t lds_per_solve)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id((int)threadIdx.x);
    char *base = smem + (size_t)wave * lds_per_solve;
    for (;;) {
        int j = 0;
        if (lane == 0) j = (int)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        j = __builtin_amdgcn_readfirstlane(j);   // lane 0's, as a scalar
        if (j >= n_jobs) return;
        run_wave_job<TE>(jobs[j], base, lane);
    }
}

hipError_t launch_search_wave(const JobDev *jobs, int32_t n_jobs, uint32_t *queue, int grid,
                              int waves_per_group, uint32_t lds_per_solve, int esz16, hipStream_t s)
{
    const uint32_t lds = lds_per_solve * (uint32_t)waves_per_group;
    hipError_t e;
    if (esz16) {
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_search_wave<uint16_t>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_search_wave<uint16_t>, dim3(grid), dim3(kWave * waves_per_group), lds, s, jobs,
                           n_jobs, queue, lds_per_solve);
    } else {
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_search_wave<int32_t>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_search_wave<int32_t>, dim3(grid), dim3(kWave * waves_per_group), lds, s, jobs,
                           n_jobs, queue, lds_per_solve);
    }
    return hipGetLastError();
}

// Test hook: every slot's key for a given state on the wave schedule's
// evaluation (the constrained model included), and the minimum.
template <typename TE>
__global__ void __launch_bounds__(64) k_debug_keys_wave(const JobDev *jp, const int32_t *off,
                                                       const int32_t *seq, const int32_t *tabu_until,
                                                       int32_t t, int64_t cur, int64_t best, uint64_t *keys)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const JobDev &J = *jp;
    const InstDev &I = *J.inst;
    const int lane = threadIdx.x;
    const WLay ly = wave_layout(I.M, I.V, I.R, I.Cs, (int)sizeof(TE), I.T2 != nullptr);
    const W<TE> c = make_w<TE>(smem, ly, I);
    const int M = c.M, V = c.V;
    if (stage(I, c, lane) != AT_OK) {
        if (lane == 0) keys[n_slots(M, V)] = kKeyNone;
        return;
    }
    for (int i = lane; i < M; i += kWave) c.seq[i] = seq[i];
    for (int v = lane; v <= V; v += kWave) c.off[v] = off[v];
    for (int k = lane; k < M * V; k += kWave) {
        const int m = k / V, v = k - m * V;
        c.tabu[v * M + m] = tabu_until[k] + 1;
    }
    wsync();
    for (int v = lane; v < V; v += kWave)
        for (int i = c.off[v]; i < c.off[v + 1]; ++i) { c.rt[i] = v; c.pof[c.seq[i]] = i; c.rof[c.seq[i]] = v; }
    wsync();
    prep(c, M, lane);
    int thr = INT32_MIN;
    if (J.aspiration) {
        const int64_t g = best - cur;
        thr = g < (int64_t)INT32_MIN ? INT32_MIN : (int)g;
    }
    const uint64_t k = wmin(eval_best(c, lane, t, thr, J.variant == AT_TABU, keys));
    if (lane == 0) keys[n_slots(M, V)] = k;
}

hipError_t launch_debug_keys_wave(const JobDev *job, const int32_t *off, const int32_t *seq,
                                  const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
                                  uint64_t *keys, uint32_t lds_bytes, int esz16, hipStream_t s)
{
    hipError_t e;
    if (esz16) {
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_debug_keys_wave<uint16_t>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_debug_keys_wave<uint16_t>, dim3(1), dim3(kWave), lds_bytes, s, job, off, seq,
                           tabu_until, t, cur, best, keys);
    } else {
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_debug_keys_wave<int32_t>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_debug_keys_wave<int32_t>, dim3(1), dim3(kWave), lds_bytes, s, job, off, seq,
                           tabu_until, t, cur, best, keys);
    }
    return hipGetLastError();
}

}  // namespace at
