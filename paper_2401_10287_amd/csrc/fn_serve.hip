// fn_serve.hip -- continuous batching of VMC jobs on one GPU.
//
// A job is: B walkers of one system (atom or ion) with its own parameters,
// n_steps Metropolis-Hastings moves (Electron Sampler section of the paper)
// and the energy estimate of Eq. 1 over its walkers (local energies of Eq. 2).
// The server keeps every admitted job's walkers, log|psi| and workspace in a
// caller-provided device arena (the job's HBM footprint), admits queued jobs
// in arrival order as soon as their footprint fits and a slot (stream) is
// free -- a job that does not fit yet may be passed by later, smaller jobs a
// bounded number of times, after which admission waits for it -- and
// advances every running job by one quantum of Metropolis steps per
// scheduler step, so the work of different jobs overlaps on the device.
// The library allocates nothing: the arena, the streams and the pinned host
// buffer the results land in are the caller's; completion is read with
// stream queries (each stream runs one job at a time).
// A job's arithmetic does not depend on what else runs: each job draws its
// random numbers from its own (seed, stream_id) counter space and uses its own
// workspace, so results are identical alone and in any mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fnvmc.h"
#include "fn_internal.h"
#include "fn_kernels.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// mean, variance (1/B), standard error of e_loc and the acceptance rate
__global__ __launch_bounds__(1024) void k_job_stats(const double *e, const int32_t *acc, int64_t B, int32_t n_steps,
                                                    double *out)
{
    __shared__ double red[2][16];
    __shared__ double s_mean;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double se = 0.0, sa = 0.0;
    for (int64_t p = tid; p < B; p += blockDim.x) { se += e[p]; sa += acc[p]; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) { se += __shfl_xor(se, off, 64); sa += __shfl_xor(sa, off, 64); }
    if (lane == 0) { red[0][wv] = se; red[1][wv] = sa; }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { a += red[0][q]; b += red[1][q]; }
        s_mean = a / (double)B;
        out[3] = n_steps > 0 ? b / ((double)B * n_steps) : 0.0;
    }
    __syncthreads();
    const double mean = s_mean;
    double sv = 0.0;
    for (int64_t p = tid; p < B; p += blockDim.x) { const double d = e[p] - mean; sv += d * d; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sv += __shfl_xor(sv, off, 64);
    __syncthreads();
    if (lane == 0) red[0][wv] = sv;
    __syncthreads();
    if (tid == 0) {
        double v = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v += red[0][q];
        v /= (double)B;
        out[0] = mean; out[1] = v; out[2] = sqrt(v / (double)B);
    }
}

__global__ void k_zero_i32(int32_t *p, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) p[q] = 0;
}

constexpr size_t AL = 256;
size_t alup(size_t v) { return (v + AL - 1) / AL * AL; }

// first-fit allocator over [0, size) of the arena, 256-byte granules
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t n) { size = n / AL * AL; free_.clear(); if (size) free_[0] = size; }
    bool alloc(size_t n, size_t &off)
    {
        n = alup(n);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = alup(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
        }
    }
    size_t free_bytes() const { size_t t = 0; for (auto &kv : free_) t += kv.second; return t; }
    size_t largest_free() const { size_t t = 0; for (auto &kv : free_) t = kv.second > t ? kv.second : t; return t; }
};

struct Job {
    int64_t id;
    fn_config cfg;
    std::vector<double> nuc_xyz, nuc_z;
    const void *theta;
    const double *x0;
    int64_t B;
    int32_t n_steps, done_steps = 0;
    double sigma;
    uint64_t seed;
    uint32_t stream_id;
    int32_t state = 0;        // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
    int32_t bypassed = 0;     // times a later job was admitted ahead of it
    int slot = -1;
    size_t off = 0, bytes = 0, ws_bytes = 0;
    size_t o_x, o_lp, o_acc, o_e, o_stats, o_ws;
    bool finishing = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double res[4] = {0, 0, 0, 0};
    std::string err;
};

struct Slot {
    hipStream_t stream;
    double *host_res;         // the caller's pinned [4]
    int64_t job = -1;
};

}  // namespace

struct fn_server {
    std::mutex mu;
    char *arena_base;
    Arena arena;
    std::vector<Slot> slots;
    int32_t quantum;
    std::map<int64_t, Job> jobs;
    std::deque<int64_t> queue;
    int32_t max_bypass;
    int64_t next_id = 0;
    std::string err;
};

namespace {

thread_local std::string g_serr;

fn_status sfail(fn_status st, const std::string &m)
{
    g_serr = m;
    return st;
}

size_t job_layout(Job &j)
{
    const int64_t B = j.B;
    const int n3 = 3 * (j.cfg.n_up + j.cfg.n_down);
    size_t ws = fn_workspace_bytes(&j.cfg, B, FN_OP_METROPOLIS);
    size_t ws2 = fn_workspace_bytes(&j.cfg, B, FN_OP_LOCAL_ENERGY);
    size_t ws3 = fn_workspace_bytes(&j.cfg, B, FN_OP_LOG_PSI);
    if (!ws || !ws2 || !ws3) return 0;
    if (ws2 > ws) ws = ws2;
    if (ws3 > ws) ws = ws3;
    size_t o = 0;
    j.o_x = o; o += alup((size_t)B * n3 * 8);
    j.o_lp = o; o += alup((size_t)B * 8);
    j.o_acc = o; o += alup((size_t)B * 4);
    j.o_e = o; o += alup((size_t)B * 8);
    j.o_stats = o; o += alup(4 * 8);
    j.o_ws = o; o += alup(ws);
    j.ws_bytes = ws;
    return o;
}

// enqueue the job's next quantum (or its energy estimate) on its stream
fn_status advance(fn_server *s, Job &j)
{
    Slot &sl = s->slots[j.slot];
    char *base = s->arena_base + j.off;
    double *x = (double *)(base + j.o_x), *lp = (double *)(base + j.o_lp), *e = (double *)(base + j.o_e);
    int32_t *acc = (int32_t *)(base + j.o_acc);
    void *ws = base + j.o_ws;
    fn_status r = FN_OK;
    if (j.done_steps < j.n_steps) {
        const int32_t q = j.n_steps - j.done_steps < s->quantum ? j.n_steps - j.done_steps : s->quantum;
        r = vmc_metropolis_step(&j.cfg, j.theta, x, lp, j.B, q, j.sigma, j.seed, (uint64_t)j.done_steps, j.stream_id,
                                acc, ws, j.ws_bytes, sl.stream);
        j.done_steps += q;
    } else {
        r = fn_local_energy(&j.cfg, j.theta, x, j.B, e, nullptr, nullptr, ws, j.ws_bytes, sl.stream);
        if (r == FN_OK) {
            double *st = (double *)(base + j.o_stats);
            hipLaunchKernelGGL(k_job_stats, dim3(1), dim3(1024), 0, sl.stream, e, acc, j.B, j.n_steps, st);
            if (hipMemcpyAsync(sl.host_res, st, 4 * sizeof(double), hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
                r = sfail(FN_EHIP, "result copy failed");
        }
        j.finishing = true;
    }
    if (r != FN_OK) {
        j.err = fn_last_error();
        return r;
    }
    return FN_OK;
}

fn_status admit(fn_server *s, Job &j, int slot)
{
    size_t off;
    if (!s->arena.alloc(j.bytes, off)) return FN_ENOMEM;
    j.off = off;
    j.slot = slot;
    j.state = 1;
    j.t_admit = now_s();
    Slot &sl = s->slots[slot];
    sl.job = j.id;
    char *base = s->arena_base + off;
    const int n3 = 3 * (j.cfg.n_up + j.cfg.n_down);
    if (hipMemcpyAsync(base + j.o_x, j.x0, (size_t)j.B * n3 * 8, hipMemcpyDeviceToDevice, sl.stream) != hipSuccess)
        return sfail(FN_EHIP, "walker copy failed");
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((j.B + 255) / 256)), dim3(256), 0, sl.stream,
                       (int32_t *)(base + j.o_acc), j.B);
    fn_status r = fn_log_psi(&j.cfg, j.theta, (double *)(base + j.o_x), j.B, (double *)(base + j.o_lp), nullptr,
                             base + j.o_ws, j.ws_bytes, sl.stream);
    if (r != FN_OK) { j.err = fn_last_error(); return r; }
    return advance(s, j);
}

void retire(fn_server *s, Job &j, int32_t state)
{
    Slot &sl = s->slots[j.slot];
    if (state != 2) (void)hipStreamSynchronize(sl.stream);   // nothing may still use the arena block
    if (state == 2)
        for (int q = 0; q < 4; ++q) j.res[q] = sl.host_res[q];
    j.state = state;
    j.t_done = now_s();
    s->arena.release(j.off, j.bytes);
    sl.job = -1;
}

}  // namespace

extern "C" {

size_t fn_server_job_bytes(const fn_config *cfg, int64_t B)
{
    if (!cfg || B <= 0) return 0;
    Job j;
    j.cfg = *cfg;
    j.B = B;
    return alup(job_layout(j));
}

fn_status fn_server_create(void *arena, size_t arena_bytes, void *const *streams, int32_t n_streams,
                           int32_t quantum_steps, double *host_results, fn_server **out)
{
    if (!arena || !streams || n_streams < 1 || !out || quantum_steps < 1 || !host_results)
        return sfail(FN_EINVAL, "invalid server arguments");
    if ((uintptr_t)arena % AL) return sfail(FN_EINVAL, "arena must be 256-byte aligned");
    fn_server *s = new fn_server();
    s->arena_base = (char *)arena;
    s->arena.init(arena_bytes);
    s->quantum = quantum_steps;
    s->max_bypass = 2 * n_streams;
    for (int i = 0; i < n_streams; ++i) {
        Slot sl;
        sl.stream = (hipStream_t)streams[i];
        sl.host_res = host_results + 4 * i;
        s->slots.push_back(sl);
    }
    *out = s;
    return FN_OK;
}

fn_status fn_server_submit(fn_server *s, const fn_config *cfg, const void *theta, const double *x0, int64_t B,
                           int32_t n_steps, double sigma, uint64_t seed, uint32_t stream_id, int64_t *job)
{
    if (!s || !cfg || !theta || !x0 || B <= 0 || n_steps < 0 || !job) return sfail(FN_EINVAL, "invalid job");
    std::lock_guard<std::mutex> lk(s->mu);
    Job j;
    j.cfg = *cfg;
    j.nuc_xyz.assign(cfg->nuc_xyz, cfg->nuc_xyz + 3 * cfg->n_nuc);
    j.nuc_z.assign(cfg->nuc_z, cfg->nuc_z + cfg->n_nuc);
    j.theta = theta;
    j.x0 = x0;
    j.B = B;
    j.n_steps = n_steps;
    j.sigma = sigma;
    j.seed = seed;
    j.stream_id = stream_id;
    j.bytes = job_layout(j);
    if (!j.bytes) return sfail(FN_EINVAL, std::string("job rejected: ") + fn_last_error());
    if (j.bytes > s->arena.size) return sfail(FN_ENOMEM, "job footprint exceeds the arena");
    j.id = s->next_id++;
    j.t_submit = now_s();
    auto it = s->jobs.emplace(j.id, std::move(j)).first;
    it->second.cfg.nuc_xyz = it->second.nuc_xyz.data();   // the job owns its copy of the nuclei
    it->second.cfg.nuc_z = it->second.nuc_z.data();
    s->queue.push_back(it->first);
    *job = it->first;
    return FN_OK;
}

fn_status fn_server_step(fn_server *s, int32_t *n_active, int32_t *n_queued)
{
    if (!s) return sfail(FN_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    // 1. progress of running jobs: retire finished ones, enqueue next quanta
    for (size_t i = 0; i < s->slots.size(); ++i) {
        Slot &sl = s->slots[i];
        if (sl.job < 0) continue;
        hipError_t q = hipStreamQuery(sl.stream);
        if (q == hipErrorNotReady) continue;
        Job &j = s->jobs[sl.job];
        if (q != hipSuccess) { j.err = hipGetErrorString(q); retire(s, j, 3); continue; }
        if (j.finishing) { retire(s, j, 2); continue; }
        if (advance(s, j) != FN_OK) retire(s, j, 3);
    }
    // 2. admission in arrival order by HBM footprint and free slot; a job
    //    that does not fit is passed by later ones that do, until it has been
    //    passed max_bypass times -- then admission waits for it
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        int slot = -1;
        for (size_t i = 0; i < s->slots.size(); ++i)
            if (s->slots[i].job < 0) { slot = (int)i; break; }
        if (slot < 0) break;
        Job &j = s->jobs[*it];
        fn_status r = admit(s, j, slot);
        if (r == FN_ENOMEM) {
            if (j.bypassed >= s->max_bypass) break;
            bool fits_later = false;          // count a pass only if someone behind is admitted
            for (auto jt = std::next(it); jt != s->queue.end() && !fits_later; ++jt)
                fits_later = s->jobs[*jt].bytes <= s->arena.largest_free();
            if (!fits_later) break;
            ++j.bypassed;
            ++it;
            continue;
        }
        it = s->queue.erase(it);
        if (r != FN_OK) retire(s, j, 3);
    }
    int32_t act = 0;
    for (auto &sl : s->slots) act += sl.job >= 0;
    if (n_active) *n_active = act;
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return FN_OK;
}

fn_status fn_server_result(fn_server *s, int64_t job, fn_job_result *out)
{
    if (!s || !out) return sfail(FN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return sfail(FN_EINVAL, "unknown job");
    const Job &j = it->second;
    out->state = j.state;
    out->mean = j.res[0];
    out->variance = j.res[1];
    out->std_error = j.res[2];
    out->acceptance = j.res[3];
    out->submit_s = j.t_submit;
    out->admit_s = j.t_admit;
    out->done_s = j.t_done;
    out->footprint_bytes = (int64_t)j.bytes;
    return FN_OK;
}

fn_status fn_server_cancel(fn_server *s, int64_t job)
{
    if (!s) return sfail(FN_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return sfail(FN_EINVAL, "unknown job");
    Job &j = it->second;
    if (j.state == 0) {
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (*q == job) { s->queue.erase(q); break; }
        j.state = 4;
        j.t_done = now_s();
    } else if (j.state == 1) {
        retire(s, j, 4);              // waits for the job's enqueued quantum, then frees its slot and memory
    }
    return FN_OK;
}

fn_status fn_server_memory(fn_server *s, size_t *free_bytes, size_t *arena_bytes)
{
    if (!s || !free_bytes || !arena_bytes) return sfail(FN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *free_bytes = s->arena.free_bytes();
    *arena_bytes = s->arena.size;
    return FN_OK;
}

fn_status fn_server_destroy(fn_server *s)
{
    if (!s) return FN_OK;
    for (auto &sl : s->slots)
        if (sl.job >= 0) (void)hipStreamSynchronize(sl.stream);
    delete s;
    return FN_OK;
}

const char *fn_server_last_error(void) { return g_serr.c_str(); }

}  // extern "C"
