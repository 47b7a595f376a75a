/*
 * atabu.h -- C ABI of the MI355X (gfx950) Tabu-search scheduler for
 * base-returning air-ambulance routes (Tassone & Choudhury, "Algorithms for
 * Optimizing Fleet Scheduling of Air Ambulances", arXiv 2002.11710).
 *
 * Problem (Section 3 of the paper): M missions, each a pickup location and a
 * delivery location, are to be flown by V vehicles; every vehicle starts and
 * ends at its own base and flies its missions in order, going from one
 * mission's delivery to the next mission's pickup.  The objective (Eq (2)) is
 * the total flight time, each mission's loaded leg included.  Times come from
 * the haversine distance over the vehicle speed (Eq (1)).
 *
 * Method (Section 4): a greedy start (Algorithm 1), then neighbourhood search
 * (Algorithm 2) or Tabu search (Algorithm 3).  Here every iteration scores every
 * relocate move (a mission to any gap of any route, Figure 2) and every swap of
 * two missions, masks moves that put a mission back into a vehicle it left
 * less than `tenure` iterations ago unless they beat the best objective found,
 * picks the smallest (delta, move index) and applies it.  All iterations of a
 * solve run inside one kernel launch.
 *
 * Conventions for every function below:
 *   - Return 0 (AT_OK) on success, a negative AT_E* code otherwise; the text of
 *     the last error of the calling thread is at_last_error().
 *   - "device" pointers are HIP device memory of the current device (for
 *     example torch CUDA tensors); "host" pointers are ordinary memory.  The
 *     caller owns every buffer; the library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that return
 *     host scalars synchronise that stream before they return.
 *   - Integers are int32 unless stated; objectives are int64 seconds.
 *   - Inputs are checked before any search kernel runs; a bad input returns an
 *     error and leaves outputs untouched.
 */
#ifndef ATABU_H
#define ATABU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AT_OK 0
#define AT_EINVAL (-1)   /* bad size, index, pickup == delivery, bad parameter */
#define AT_ERANGE (-2)   /* a travel time outside [0, 2^23), or too many move slots */
#define AT_ENOMEM (-3)   /* workspace too small, or a request over the memory budget */
#define AT_EAGAIN (-4)   /* result not ready yet (serving) */
#define AT_EDEVICE (-5)  /* a HIP error or a device-side failure */
#define AT_EINFEAS (-6)  /* Algorithm 1 found no feasible start (constrained model) */

#define AT_TABU 0        /* Tabu search (Algorithm 3) */
#define AT_NS 1          /* neighbourhood search (Algorithm 2): stops at a local optimum */

/* Schedules (at_params.schedule). */
#define AT_SCHED_AUTO 0
#define AT_SCHED_WG 1    /* one workgroup per solve, the whole state in LDS */
#define AT_SCHED_MULTI 2 /* several workgroups per solve, state replicated in each one's LDS */
#define AT_SCHED_GLOBAL 3 /* several workgroups per solve, state in HBM (large instances) */
#define AT_SCHED_WAVE 4  /* one wavefront per solve, the whole state in LDS (small instances,
                            the constrained model and the sweep form) */

/* Forms of the search (at_params.form). */
#define AT_FORM_BEST 0   /* every iteration scores the whole neighbourhood and applies the best */
#define AT_FORM_SWEEP 1  /* Algorithms 2 and 3 as printed: bases in turn, each base's missions in
                            turn, each mission moved to its best strictly better place in
                            another base (WAVE schedule only) */

/* One instance.  Locations are numbered 0..n_locs-1; the travel matrix gives
 * integer seconds, travel[i*n_locs + j] = time from location i to location j
 * (for example the output of at_build_travel).  Mission m is flown from
 * pickup[m] to delivery[m]; vehicle v starts and ends at vehicle_loc[v].
 * Limits: 1 <= n_locs <= 65535, 0 <= n_missions <= 65535, 1 <= n_vehicles
 * <= 65535, pickup != delivery, every travel time in [0, 2^23), and
 * M*(M+V) + M*(M-1)/2 < 2^32.
 *
 * The constrained model of Section 3 (Eqs (7)-(10)) is switched on field by
 * field (all NULL / 0: the unconstrained model, every move feasible):
 *   travel_plane, vehicle_type: a second matrix for planes (Eq (1) at the
 *     plane speed) and each vehicle's type (0 helicopter: `travel`; 1 plane:
 *     `travel_plane`); each route's flights, loaded legs included, are timed
 *     in its vehicle's matrix (Eq (2) with l = b_k);
 *   deadline: the time (seconds from the start, >= 0) by which mission m's
 *     vehicle must reach its delivery point; the vehicle then waits there
 *     until that time before it flies on (Eqs (8)-(9)); every vehicle leaves
 *     its base at 0 and must be back by `horizon`;
 *   heli_only: 1 for a mission only a helicopter may fly (Eq (10));
 *   flight_limit > 0: a route's flight time, waiting excluded, is at most
 *     this (Eq (7)).
 * A move whose result breaks a constraint is not a move.  The constrained
 * model runs on the WAVE schedule only, with at most 1024 missions and 256
 * vehicles, and its greedy start is Algorithm 1 with its checks (see
 * at_params); a solve without a feasible start ends with status AT_EINFEAS. */
typedef struct at_instance {
    int32_t n_locs;
    const int32_t *travel;       /* device, n_locs*n_locs, row-major */
    int32_t n_missions;
    const int32_t *pickup;       /* device, n_missions */
    const int32_t *delivery;     /* device, n_missions */
    int32_t n_vehicles;
    const int32_t *vehicle_loc;  /* device, n_vehicles */
    const int32_t *travel_plane; /* device, n_locs*n_locs, or NULL (one matrix) */
    const int32_t *vehicle_type; /* device, n_vehicles (0 or 1), or NULL (all 0) */
    const int32_t *deadline;     /* device, n_missions, or NULL (no time limits) */
    const int32_t *heli_only;    /* device, n_missions (0 or 1), or NULL (none) */
    int32_t flight_limit;        /* seconds of flight per vehicle; <= 0: no limit */
    int32_t horizon;             /* seconds; used with deadline (> 0) */
} at_instance;

typedef struct at_params {
    int32_t variant;        /* AT_TABU or AT_NS */
    int32_t tenure;         /* >= 0: iterations a mission may not re-enter the vehicle it left */
    int32_t max_iters;      /* >= 0 */
    int32_t aspiration;     /* 1: a tabu move is allowed when it beats the best objective */
    uint64_t restart_seed;  /* 0: greedy start in mission order; else a SplitMix64-driven
                               Fisher-Yates order of the missions */
    int32_t trace;          /* 1: write the per-iteration trace into at_result */
    int32_t schedule;       /* AT_SCHED_* (AUTO picks by size) */
    int32_t n_groups;       /* workgroups per solve for MULTI/GLOBAL (0 = auto) */
    int32_t block;          /* threads per workgroup: 0 = auto, else 256, 512 or 1024 (the
                               HBM-resident schedule uses at most 512) */
    int32_t chunk;          /* partner positions per swap work unit: 0 = auto, else 4, 8,
                               16, 32 or 64 (relocate units take twice as many gaps, at most
                               64) */
    int32_t form;           /* AT_FORM_BEST or AT_FORM_SWEEP */
} at_params;

/* The sweep form (AT_FORM_SWEEP), Algorithm 2 (AT_NS) or 3 (AT_TABU) as
 * printed: passes over the vehicles, each vehicle's missions (those on it
 * when its turn begins) in turn; each mission moves to the gap of another
 * vehicle with the smallest cost change if that change is negative (the
 * first such gap in vehicle then position order on ties; compatible,
 * feasible, and for Tabu not listed); Tabu lists (mission, vehicle left) for
 * tenure - 1 further turns.  Passes end when one moves nothing or after
 * max_iters turns.  With restart_seed != 0 the vehicle order of every pass and
 * the mission order of every vehicle's turn are Fisher-Yates orders drawn in
 * that sequence from SplitMix64(restart_seed).  Results: one trace record per
 * turn (the relocate slot index, or 0xFFFFFFFF when the mission stays; flags
 * 0); the best solution is the final one; iters_done = turns run; best_iter =
 * the last turn that moved a mission.
 *
 * The greedy start of the constrained model (Algorithm 1): helicopter-only
 * missions first, then the others, each group by deadline (ties: mission id,
 * or rank in the SplitMix64(restart_seed) Fisher-Yates order); each mission is
 * appended to the vehicle where it fits at the least added flight time (ties:
 * lowest vehicle); where it fits nowhere, one Algorithm 2 sweep over the
 * missions placed so far, then one more try, then AT_EINFEAS. */

/* Results of one solve.  Arrays are device memory supplied by the caller;
 * scalars are written by the library (host).  The routes are the best
 * solution seen (the greedy start counts, best_iter = -1); final_off and
 * final_seq, when given, receive the routes the search ends on, in the same
 * layout.  Route v holds
 * missions route_seq[route_off[v] .. route_off[v+1]) in flying order;
 * route_of[m] is the vehicle of mission m.  Trace record t (t < iters_done):
 * the slot index of the applied move (0xFFFFFFFF when no move exists), its
 * delta, the objective after it, and flags: bit0 swap move, bit1 the move was
 * tabu but allowed by aspiration, bit2 every allowed move was tabu and the best
 * tabu move was taken.  Slot indices: relocating mission m into gap G is
 * m*(M+V) + G, where the gaps of vehicle v are numbered G = (missions on
 * vehicles before v) + v + g, g = 0..(missions on v), gap g lying before the
 * g-th mission of the route (g = missions on v: before the return to base);
 * swapping missions a < b is M*(M+V) + a*M - a*(a+1)/2 + (b - a - 1). */
typedef struct at_result {
    int32_t *route_off;     /* device, V+1 */
    int32_t *route_seq;     /* device, M */
    int32_t *route_of;      /* device, M (may be NULL) */
    int32_t *final_off;     /* device, V+1 (may be NULL): routes after the last iteration */
    int32_t *final_seq;     /* device, M (NULL when final_off is NULL) */
    uint32_t *tr_move;      /* device, max_iters (NULL when trace == 0) */
    int32_t *tr_delta;      /* device, max_iters */
    int64_t *tr_obj;        /* device, max_iters */
    uint8_t *tr_flags;      /* device, max_iters */
    int64_t best_obj;       /* out */
    int64_t final_obj;      /* out: objective after the last iteration */
    int32_t iters_done;     /* out: iterations run (NS: moves applied) */
    int32_t best_iter;      /* out */
    int32_t status;         /* out: AT_OK or the solve's error code */
    float search_ms;        /* out: duration of the search launch that ran this solve, in ms,
                               from HIP events recorded on `stream` around it (a batch shares
                               one launch per kernel class; every solve of it reports that) */
} at_result;

/* Eq (1) (Section 3 of the paper): travel-time matrix of n points, on the
 * host.  lat_deg, lon_deg: host, n doubles (degrees: latitude and longitude
 * are the paper's row and column coordinates phi, psi); travel: host, n*n
 * int32 written row-major, travel[i*n + j] = round-half-away-from-zero of
 * 2*6371*asin(sqrt(min(1, a))) * 3600 / speed_kmh seconds with
 * a = sin^2((phi_j - phi_i)/2) + cos(phi_i) cos(phi_j) sin^2((psi_j - psi_i)/2),
 * in FP64 with the system libm, without contraction, in that order.  Every
 * ordered pair is computed (nothing is mirrored); the diagonal is 0.
 * AT_EINVAL if n < 1, n > 65535, a pointer is null or speed_kmh is not a
 * positive finite number; AT_ERANGE if a time does not fit int32 (travel is
 * then unspecified).  Synchronous; touches no device. */
int at_build_travel(int32_t n, const double *lat_deg, const double *lon_deg, double speed_kmh,
                    int32_t *travel);

/* The same matrix computed on the device, one thread per ordered pair: lat_deg,
 * lon_deg and travel are device pointers; asynchronous on `stream`.  Its
 * sin/cos/asin/sqrt are the device math library's, which may round a
 * different way than the host libm in rare cases, so a time within an ulp of a
 * half second could differ by one from at_build_travel; a time above INT32_MAX
 * is written as INT32_MAX (the solve then rejects it with AT_ERANGE).  Same
 * argument errors as at_build_travel. */
int at_build_travel_device(int32_t n, const double *lat_deg, const double *lon_deg,
                           double speed_kmh, int32_t *travel, void *stream);

/* Bytes of device workspace at_solve_batch needs for these instances and
 * parameters (n_inst entries each, n_restarts solves per instance).  0 on bad
 * arguments. */
size_t at_workspace_size(int32_t n_inst, const at_instance *insts, const at_params *params,
                         int32_t n_restarts);

/* Solve one instance: greedy start, then the search (Sections 4.1-4.3).
 * ws: device workspace of ws_bytes >= at_workspace_size(1, inst, params, 1).
 * Blocking on `stream`; fills out's device arrays and host scalars. */
int at_solve(const at_instance *inst, const at_params *params, void *ws, size_t ws_bytes,
             void *stream, at_result *out);

/* at_solve for callers that cannot allocate memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation, code being
 * prepared for graph capture).  Same instance, parameters, results and
 * errors as at_solve, without a workspace argument: the workspace is a fixed
 * 64 MiB device array inside the library (one per device, created when the
 * library's code is loaded on that device and held until the process ends).
 * Nothing is allocated on the device or in pinned host memory, and no stream
 * or event is created; search_ms is reported as 0.  A solve whose workspace
 * (at_workspace_size(1, inst, params, 1)) exceeds 64 MiB returns AT_ENOMEM
 * before touching the device (the 10 000-mission, 2200-location stress
 * instance needs 57 MiB; a 16 000-mission instance on 4300 locations would
 * need over 200 MiB).  The array keeps the last call's contents and every call sets up
 * what it reads; calls on one device share it, so calls from several host
 * threads are serialised by a per-device lock (each is blocking on its
 * stream), and work on the device that overlaps a call must not use it. */
int at_solve_noalloc(const at_instance *inst, const at_params *params, void *stream,
                     at_result *out);

/* Solve n_inst instances x n_restarts restarts.  params[i] applies to
 * instance i; restart r of instance i starts from restart_seed 0 when r == 0
 * and from params[i].restart_seed + r otherwise.  out has n_inst*n_restarts
 * entries, solve (i, r) at out[i*n_restarts + r].  Every solve gives the same
 * result as the corresponding at_solve.  Blocking on `stream`. */
int at_solve_batch(int32_t n_inst, const at_instance *insts, const at_params *params,
                   int32_t n_restarts, void *ws, size_t ws_bytes, void *stream,
                   at_result *out);

/* Test hook: the 64-bit key of every move slot for a given state, one move at
 * a time (bit63 tabu-and-not-aspirated, bits 62..32 delta + 2^30, bits 31..0
 * slot index; UINT64_MAX for a slot that is not a move), followed by the
 * minimum key the search's own evaluation finds for that state.  route_off
 * (V+1), route_seq (M), tabu_until (M*V, entry m*V+v = last iteration at which
 * mission m may not enter vehicle v, -1 = never) and keys_out
 * (M*(M+V) + M*(M-1)/2 + 1 entries) are device pointers.  t is the iteration,
 * cur and best the current and best objectives.  Blocking. */
int at_debug_eval_moves(const at_instance *inst, const at_params *params,
                        const int32_t *route_off, const int32_t *route_seq,
                        const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
                        uint64_t *keys_out, void *ws, size_t ws_bytes, void *stream);

/* Serving with continuous batching.  A server owns device memory up to
 * hbm_budget_bytes and up to max_slots concurrent solves.  Submitted requests
 * wait until a slot and enough budget are free, then join the solves already
 * on the GPU: every launch advances each resident solve at least `chunk_iters`
 * iterations or all that remain.  Solves short enough to finish within the
 * launch on one workgroup run to the end, taken from a queue by the launch's
 * worker workgroups; longer ones get workgroups of their own for at least
 * chunk_iters iterations, so requests that arrive while others run start
 * within one launch.  (When the resident solves differ in entry or tabu width,
 * each launch instead runs chunk_iters iterations of every solve, and a
 * one-workgroup solve with S move slots per iteration, S < 2^20,
 * floor(2^20 / S) times as many.)  Each request's result is the same as
 * at_solve's.
 * `stream` is the caller's: requests are admitted (their instance arrays read)
 * and results copied out on it; the solves themselves run on an internal
 * stream of default priority, so a poll never waits for the launch in flight.
 * at_server_submit returns a ticket; the instance's device arrays are read
 * when the request is admitted, so the caller keeps them valid until
 * at_server_poll has returned the result;
 * at_server_poll returns AT_OK with the result when done (out's arrays are
 * device memory of the caller, filled on `stream` and complete on return),
 * AT_EAGAIN while pending;
 * at_server_completed writes up to `capacity` tickets of requests that are
 * done and not yet polled, each once, in the order they finished (*n_out of
 * them), so a caller polls only those;
 * at_server_progress drives the device (call it from one thread, in a loop);
 * at_server_destroy waits for running work and frees everything. */
int at_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t chunk_iters,
                     void *stream, void **server);
int at_server_submit(void *server, const at_instance *inst, const at_params *params,
                     uint64_t *ticket);
int at_server_progress(void *server, int32_t *n_active);
int at_server_poll(void *server, uint64_t ticket, at_result *out);
int at_server_completed(void *server, uint64_t *tickets, int32_t capacity, int32_t *n_out);
int at_server_destroy(void *server);

/* Release what the library holds between calls: the internal streams on
 * which the one-workgroup launches of a batch's different size classes run
 * concurrently (created on first use, each synchronised before it is
 * destroyed).  Optional; call it with no other library call in flight, for
 * example before the process exits, so that nothing of the library is left
 * for the runtime's exit-time teardown.  A later call creates them again.
 * Servers are released by at_server_destroy, not here.  AT_EDEVICE if a
 * synchronisation or destruction fails. */
int at_shutdown(void);

/* Thread-local text of the last error returned on this thread. */
const char *at_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ATABU_H */
