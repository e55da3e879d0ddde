// fn_serve.hip -- continuous batching of VMC jobs on one GPU.
//
// A job is: B walkers of one system (atom or ion) with its own parameters,
// n_steps Metropolis-Hastings moves (Electron Sampler section of the paper)
// and the energy estimate of Eq. 1 over its walkers (local energies of Eq. 2).
// Admission works in gangs: a queued job is admitted together with later
// queued jobs of the same system (same configuration, parameters, step size
// and step count), up to max_gang jobs and gang_walkers walkers in total.  A
// gang's walkers, log|psi|, counters, energies and shared workspace sit in
// one block of a caller-provided device arena (its HBM footprint), and each
// quantum of Metropolis moves of all its jobs is one grouped call (one launch
// sequence over a job table) on the gang's stream, so small jobs share
// launches instead of each running a chain of small kernels alone.  Gangs
// are admitted in arrival order of their first job as soon as the block fits
// and a stream is free -- a job that does not fit yet may be passed by later
// jobs a bounded number of times, after which admission waits for it -- and
// every running gang advances by one quantum per scheduler step, so the work
// of different gangs overlaps on the device.
// The library allocates nothing: the arena, the streams and the pinned host
// buffer the results land in are the caller's; completion is read with
// stream queries (each stream runs one gang at a time).
// A job's arithmetic does not depend on what else runs: each job draws its
// random numbers from its own (seed, stream_id) counter space, every call
// takes the batch-size-independent kernel path, and the log|psi| and energy
// estimate of a job are computed over its own walkers, so results are
// identical alone, in any gang and in any mix.
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
    int32_t n_steps;
    double sigma;
    uint64_t seed;
    uint32_t stream_id;
    int32_t state = 0;        // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
    int32_t bypassed = 0;     // times a later job was admitted ahead of it
    int64_t gang = -1;
    int64_t w0 = 0;           // first walker of the job in its gang's block
    int32_t gang_jobs = 0;    // jobs in that gang
    size_t bytes = 0;         // footprint of the job alone
    double t_submit = 0, t_admit = 0, t_done = 0;
    double res[4] = {0, 0, 0, 0};
    std::string err;
};

// jobs of one system admitted together: their walkers, log|psi|, acceptance
// counters and energies sit back to back in one arena block, the Metropolis
// moves of all of them go through one grouped call per quantum, and the
// workspace is shared (calls on the gang's stream run one after another)
struct Gang {
    std::vector<int64_t> members;    // job ids in walker order
    int slot = -1;
    size_t off = 0, bytes = 0, ws_bytes = 0;
    size_t o_x = 0, o_lp = 0, o_acc = 0, o_e = 0, o_stats = 0, o_ws = 0;
    int64_t B_total = 0;
    int32_t n_steps = 0, done_steps = 0;
    bool finishing = false;
};

struct Slot {
    hipStream_t stream;
    double *host_res;         // the caller's pinned [max_gang][4]
    int64_t gang = -1;
};

}  // namespace

struct fn_server {
    std::mutex mu;
    char *arena_base;
    Arena arena;
    std::vector<Slot> slots;
    int32_t quantum;
    int32_t max_gang;
    int64_t gang_walkers;
    std::map<int64_t, Job> jobs;
    std::map<int64_t, Gang> gangs;
    std::deque<int64_t> queue;
    int32_t max_bypass;
    int64_t next_id = 0, next_gang = 0;
    std::string err;
};

namespace {

thread_local std::string g_serr;

fn_status sfail(fn_status st, const std::string &m)
{
    g_serr = m;
    return st;
}

// the small-batch split-reduction products change the summation order with
// the batch size; every server call runs without them, so a job's results do
// not depend on which gang it runs in
struct NoSplitK {
    bool prev = fn::g_splitk_suppressed;
    NoSplitK() { fn::g_splitk_suppressed = true; }
    ~NoSplitK() { fn::g_splitk_suppressed = prev; }
};

// byte layout of a gang of `walkers` in total, the largest job `bmax` and n
// jobs; 0 if the configuration is rejected
size_t gang_layout(const fn_config &cfg, int64_t walkers, int64_t bmax, int n, Gang *g)
{
    const int n3 = 3 * (cfg.n_up + cfg.n_down);
    size_t ws = fn_workspace_bytes(&cfg, walkers, FN_OP_METROPOLIS);
    const size_t ws2 = fn_workspace_bytes(&cfg, bmax, FN_OP_LOCAL_ENERGY);
    const size_t ws3 = fn_workspace_bytes(&cfg, bmax, FN_OP_LOG_PSI);
    if (!ws || !ws2 || !ws3) return 0;
    if (ws2 > ws) ws = ws2;
    if (ws3 > ws) ws = ws3;
    Gang t;
    size_t o = 0;
    t.o_x = o; o += alup((size_t)walkers * n3 * 8);
    t.o_lp = o; o += alup((size_t)walkers * 8);
    t.o_acc = o; o += alup((size_t)walkers * 4);
    t.o_e = o; o += alup((size_t)walkers * 8);
    t.o_stats = o; o += alup((size_t)n * 4 * 8);
    t.o_ws = o; o += alup(ws);
    t.ws_bytes = ws;
    t.bytes = alup(o);
    if (g) {
        g->o_x = t.o_x; g->o_lp = t.o_lp; g->o_acc = t.o_acc; g->o_e = t.o_e; g->o_stats = t.o_stats;
        g->o_ws = t.o_ws; g->ws_bytes = t.ws_bytes; g->bytes = t.bytes;
    }
    return t.bytes;
}

// jobs that may share a gang: one system (identical configuration and
// nuclei), one parameter vector, one step size and step count
bool same_system(const Job &a, const Job &b)
{
    const fn_config &p = a.cfg, &q = b.cfg;
    if (a.theta != b.theta || a.sigma != b.sigma || a.n_steps != b.n_steps) return false;
    if (p.n_nuc != q.n_nuc || p.n_up != q.n_up || p.n_down != q.n_down || p.n_layers != q.n_layers || p.w1 != q.w1 ||
        p.w2 != q.w2 || p.n_det != q.n_det || p.precision != q.precision || p.envelope != q.envelope)
        return false;
    return a.nuc_xyz == b.nuc_xyz && a.nuc_z == b.nuc_z;
}

Job &job_at(fn_server *s, int64_t id) { return s->jobs.find(id)->second; }

void finish_job(Job &j, int32_t state, const double *res)
{
    if (j.state != 1) return;             // a member cancelled while its gang ran keeps its state
    if (res)
        for (int q = 0; q < 4; ++q) j.res[q] = res[q];
    j.state = state;
    j.t_done = now_s();
}

// enqueue the gang's next quantum (or its energy estimates) on its stream
fn_status advance(fn_server *s, Gang &g)
{
    Slot &sl = s->slots[g.slot];
    char *base = s->arena_base + g.off;
    double *x = (double *)(base + g.o_x), *lp = (double *)(base + g.o_lp), *e = (double *)(base + g.o_e);
    double *st = (double *)(base + g.o_stats);
    int32_t *acc = (int32_t *)(base + g.o_acc);
    void *ws = base + g.o_ws;
    const Job &j0 = job_at(s, g.members[0]);
    const int n3 = 3 * (j0.cfg.n_up + j0.cfg.n_down);
    NoSplitK nosplit_;
    fn_status r = FN_OK;
    if (g.done_steps < g.n_steps) {
        const int32_t q = g.n_steps - g.done_steps < s->quantum ? g.n_steps - g.done_steps : s->quantum;
        fn_group_job tab[FN_MAX_GROUP_JOBS];
        for (size_t k = 0; k < g.members.size(); ++k) {
            const Job &j = job_at(s, g.members[k]);
            tab[k].walker0 = j.w0;
            tab[k].B = j.B;
            tab[k].seed = j.seed;
            tab[k].step0 = (uint64_t)g.done_steps;
            tab[k].stream_id = j.stream_id;
        }
        r = vmc_metropolis_step_group(&j0.cfg, j0.theta, tab, (int32_t)g.members.size(), x, lp, acc, g.B_total, q,
                                      j0.sigma, ws, g.ws_bytes, sl.stream);
        g.done_steps += q;
    } else {
        for (size_t k = 0; k < g.members.size() && r == FN_OK; ++k) {
            const Job &j = job_at(s, g.members[k]);
            r = fn_local_energy(&j.cfg, j.theta, x + j.w0 * n3, j.B, e + j.w0, nullptr, nullptr, ws, g.ws_bytes,
                                sl.stream);
            if (r == FN_OK)
                hipLaunchKernelGGL(k_job_stats, dim3(1), dim3(1024), 0, sl.stream, e + j.w0, acc + j.w0, j.B,
                                   j.n_steps, st + 4 * k);
        }
        if (r == FN_OK &&
            hipMemcpyAsync(sl.host_res, st, g.members.size() * 4 * sizeof(double), hipMemcpyDeviceToHost,
                           sl.stream) != hipSuccess)
            r = sfail(FN_EHIP, "result copy failed");
        g.finishing = true;
    }
    return r;
}

void retire(fn_server *s, int64_t gid, int32_t state, const std::string &why)
{
    Gang &g = s->gangs.find(gid)->second;
    Slot &sl = s->slots[g.slot];
    if (state != 2) (void)hipStreamSynchronize(sl.stream);   // nothing may still use the arena block
    for (size_t k = 0; k < g.members.size(); ++k) {
        Job &j = job_at(s, g.members[k]);
        if (state == 3 && j.state == 1) j.err = why;
        finish_job(j, state, state == 2 ? sl.host_res + 4 * k : nullptr);
    }
    s->arena.release(g.off, g.bytes);
    sl.gang = -1;
    s->gangs.erase(gid);
}

// the gang the queued job at position qi heads: it and later queued jobs of
// the same system, in queue order, up to max_gang jobs and gang_walkers
// walkers, shrunk from the back until the block fits the arena; empty if the
// job alone does not fit
std::vector<int64_t> form_gang(fn_server *s, size_t qi)
{
    const Job &h = job_at(s, s->queue[qi]);
    std::vector<int64_t> mem{h.id};
    int64_t total = h.B;
    if (s->max_gang > 1)
        for (size_t k = qi + 1; k < s->queue.size() && (int32_t)mem.size() < s->max_gang; ++k) {
            const Job &j = job_at(s, s->queue[k]);
            if (same_system(h, j) && total + j.B <= s->gang_walkers) {
                mem.push_back(j.id);
                total += j.B;
            }
        }
    const size_t room = s->arena.largest_free();
    while (!mem.empty()) {
        int64_t walkers = 0, bmax = 0;
        for (int64_t id : mem) {
            const int64_t b = job_at(s, id).B;
            walkers += b;
            bmax = b > bmax ? b : bmax;
        }
        const size_t need = gang_layout(h.cfg, walkers, bmax, (int)mem.size(), nullptr);
        if (need && need <= room) break;
        mem.pop_back();
    }
    return mem;
}

// admit the gang on `slot`: copy the walkers in, compute their log|psi| and
// enqueue the first quantum
void start_gang(fn_server *s, const std::vector<int64_t> &mem, int slot)
{
    const int64_t gid = s->next_gang++;
    Gang &g = s->gangs[gid];
    g.members = mem;
    g.slot = slot;
    int64_t bmax = 0;
    for (int64_t id : mem) {
        Job &j = job_at(s, id);
        j.w0 = g.B_total;
        j.gang = gid;
        j.gang_jobs = (int32_t)mem.size();
        j.state = 1;
        j.t_admit = now_s();
        g.B_total += j.B;
        bmax = j.B > bmax ? j.B : bmax;
    }
    for (int64_t id : mem)
        for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
            if (*it == id) { s->queue.erase(it); break; }
    const Job &j0 = job_at(s, mem[0]);
    g.n_steps = j0.n_steps;
    gang_layout(j0.cfg, g.B_total, bmax, (int)mem.size(), &g);
    s->arena.alloc(g.bytes, g.off);           // form_gang checked that it fits
    Slot &sl = s->slots[slot];
    sl.gang = gid;
    char *base = s->arena_base + g.off;
    const int n3 = 3 * (j0.cfg.n_up + j0.cfg.n_down);
    fn_status r = FN_OK;
    std::string why;
    for (int64_t id : mem) {
        const Job &j = job_at(s, id);
        if (hipMemcpyAsync(base + g.o_x + (size_t)j.w0 * n3 * 8, j.x0, (size_t)j.B * n3 * 8, hipMemcpyDeviceToDevice,
                           sl.stream) != hipSuccess) {
            r = FN_EHIP;
            why = "walker copy failed";
            break;
        }
    }
    if (r == FN_OK)
        hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((g.B_total + 255) / 256)), dim3(256), 0, sl.stream,
                           (int32_t *)(base + g.o_acc), g.B_total);
    {
        NoSplitK nosplit_;
        for (size_t k = 0; k < mem.size() && r == FN_OK; ++k) {
            const Job &j = job_at(s, mem[k]);
            r = fn_log_psi(&j.cfg, j.theta, (double *)(base + g.o_x) + j.w0 * n3, j.B,
                           (double *)(base + g.o_lp) + j.w0, nullptr, base + g.o_ws, g.ws_bytes, sl.stream);
            if (r) why = fn_last_error();
        }
    }
    if (r == FN_OK && (r = advance(s, g)) != FN_OK) why = g_serr.empty() ? fn_last_error() : g_serr;
    if (r != FN_OK) retire(s, gid, 3, why);
}

int free_slot(fn_server *s)
{
    for (size_t i = 0; i < s->slots.size(); ++i)
        if (s->slots[i].gang < 0) return (int)i;
    return -1;
}

}  // namespace

extern "C" {

size_t fn_server_job_bytes(const fn_config *cfg, int64_t B)
{
    if (!cfg || B <= 0) return 0;
    return gang_layout(*cfg, B, B, 1, nullptr);
}

fn_status fn_server_create(void *arena, size_t arena_bytes, void *const *streams, int32_t n_streams,
                           int32_t quantum_steps, int32_t max_gang, int64_t gang_walkers, double *host_results,
                           fn_server **out)
{
    if (!arena || !streams || n_streams < 1 || !out || quantum_steps < 1 || !host_results)
        return sfail(FN_EINVAL, "invalid server arguments");
    if (max_gang < 1 || max_gang > FN_MAX_GROUP_JOBS) return sfail(FN_EINVAL, "max_gang out of range 1..64");
    if (gang_walkers < 1) return sfail(FN_EINVAL, "gang_walkers < 1");
    if ((uintptr_t)arena % AL) return sfail(FN_EINVAL, "arena must be 256-byte aligned");
    fn_server *s = new fn_server();
    s->arena_base = (char *)arena;
    s->arena.init(arena_bytes);
    s->quantum = quantum_steps;
    s->max_gang = max_gang;
    s->gang_walkers = gang_walkers;
    s->max_bypass = 2 * n_streams;
    for (int i = 0; i < n_streams; ++i) {
        Slot sl;
        sl.stream = (hipStream_t)streams[i];
        sl.host_res = host_results + (size_t)4 * max_gang * i;
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
    j.bytes = gang_layout(j.cfg, B, B, 1, nullptr);
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
    // 1. progress of running gangs: retire finished ones, enqueue next quanta
    for (size_t i = 0; i < s->slots.size(); ++i) {
        Slot &sl = s->slots[i];
        if (sl.gang < 0) continue;
        hipError_t q = hipStreamQuery(sl.stream);
        if (q == hipErrorNotReady) continue;
        const int64_t gid = sl.gang;
        Gang &g = s->gangs.find(gid)->second;
        if (q != hipSuccess) { retire(s, gid, 3, hipGetErrorString(q)); continue; }
        if (g.finishing) { retire(s, gid, 2, ""); continue; }
        if (advance(s, g) != FN_OK) retire(s, gid, 3, g_serr.empty() ? fn_last_error() : g_serr);
    }
    // 2. admission in arrival order by HBM footprint and free slot, each
    //    admitted job taking later queued jobs of its system into its gang;
    //    a job that does not fit is passed by later ones that do, until it
    //    has been passed max_bypass times -- then admission waits for it
    for (;;) {
        const int slot = free_slot(s);
        if (slot < 0) break;
        bool admitted = false;
        for (size_t qi = 0; qi < s->queue.size(); ++qi) {
            Job &j = job_at(s, s->queue[qi]);
            std::vector<int64_t> mem = form_gang(s, qi);
            if (mem.empty()) {
                if (j.bypassed >= s->max_bypass) break;
                bool fits_later = false;      // count a pass only if someone behind can be admitted
                for (size_t k = qi + 1; k < s->queue.size() && !fits_later; ++k)
                    fits_later = job_at(s, s->queue[k]).bytes <= s->arena.largest_free();
                if (!fits_later) break;
                ++j.bypassed;
                continue;
            }
            start_gang(s, mem, slot);
            admitted = true;
            break;
        }
        if (!admitted) break;
    }
    int32_t act = 0;
    for (auto &kv : s->gangs)
        for (int64_t id : kv.second.members) act += job_at(s, id).state == 1;
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
    out->gang_jobs = j.gang_jobs;
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
        finish_job(j, 4, nullptr);
        const int64_t gid = j.gang;
        bool any = false;
        for (int64_t id : s->gangs.find(gid)->second.members) any |= job_at(s, id).state == 1;
        if (!any) retire(s, gid, 4, "");    // waits for the gang's enqueued work, then frees its slot and block
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
        if (sl.gang >= 0) (void)hipStreamSynchronize(sl.stream);
    delete s;
    return FN_OK;
}

const char *fn_server_last_error(void) { return g_serr.c_str(); }

}  // extern "C"
