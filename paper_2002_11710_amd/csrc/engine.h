// engine.h -- host-side pieces shared by the solve/batch API (api.hip) and the
// serving loop (server.hip): argument checks, workspace carving, instance
// preparation, schedule choice and launches.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "atabu.h"
#include "atabu_internal.h"

namespace at {

// LDS a workgroup may use on gfx950 (160 KiB), minus room for static LDS.
constexpr uint32_t kLdsLimit = 160u * 1024u - 64u;

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t al16c(size_t x) { return (x + 15) & ~(size_t)15; }

// One solve as the host plans it.
struct JobHost {
    int inst = 0;
    at_params pr{};
    uint64_t seed = 0;
    at_result out{};
    int64_t slots = 0;
    int64_t iters = 0;                // iterations this launch runs (weights shared launches)
    uint32_t lds = 0;
    int tb16 = 0, esz16 = 0, block = 256, chunk = 16, rchunk = 16, groups = 1;
    int kind = AT_SCHED_WG;           // AT_SCHED_WG, AT_SCHED_MULTI or AT_SCHED_GLOBAL
    int gk = 0, gkmax = 0;            // global schedule: missions staged per block (chosen, LDS limit)
    int dM = 0, dV = 0, dR = 0, dC = 0, desz = 4;   // instance sizes (global schedule LDS plan)
    int g0 = 0, launch = 0;           // global / multi schedules: first workgroup, launch index
    int mx = 0;                       // multi schedule: slot set in the launch
    GlobalBufs *gstate = nullptr;     // reserved HBM state (global schedule)
    bool chunked = false;             // run in chunks of iterations (serving): no wave schedule
    bool wtile = false;               // wave schedule on the one-workgroup code (unconstrained best form)
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
const char *last_error();
int check_scalars(const at_instance *in, const at_params *pr);
int tabu_bytes(const at_params &pr);
int ring_slots(const at_params &pr);
bool may_need_global(const at_instance &in, const at_params &pr);
size_t inst_bytes(const at_instance &in, bool with_t);
size_t gstate_bytes(const at_instance &in, const at_params &pr);
void carve_inst(InstDev &d, const at_instance &in, char *base, bool with_t);
void carve_gstate(GlobalBufs &g, int M, int V, int n_ring, char *base);
int prepare_enqueue(int32_t n_inst, InstDev *dev, InstDev *host, hipStream_t s);
int prepare_check(int32_t n_inst, const InstDev *host);
int prepare_instances(int32_t n_inst, InstDev *dev, std::vector<InstDev> &host, hipStream_t s);
int plan_job(JobHost &h, const InstDev &d, bool alone);
// Solves at or above this many move slots take the multi-workgroup schedule
// under AUTO when they are alone in their call (or in a small batch).
constexpr int64_t kMultiMinSlots = 20000;
constexpr int kMultiMaxGroups = 96;       // workgroups of one multi-workgroup solve (auto plan)
bool multi_eligible(const JobHost &h);
int plan_multi(JobHost &h, const InstDev &d, bool small_units = true);
int plan_multi_batch(std::vector<JobHost> &jobs, const std::vector<InstDev> &ih);
int fill_job(JobDev &j, const JobHost &h, const InstDev *dev_inst, JobScal *scal);
int upload_gstates(const std::vector<JobHost> &jobs, const std::vector<InstDev> &ih, hipStream_t s);
int launch_jobs(const std::vector<JobHost> &jobs, const std::vector<int> &order, JobDev *dj,
                Xchg *xs, hipStream_t s);
std::vector<int> order_jobs(const std::vector<JobHost> &jobs);
int assign_groups(std::vector<JobHost> &jobs, const std::vector<int> &order);
void set_block_size(JobHost &h);

}  // namespace at
