// fn_api.hip -- the C ABI of fnvmc.h: argument checks, workspace plan and
// the host-side sequence of kernels for each entry point.
//
// Forward pass over a chunk of walkers (FermiNet Model section):
//   features -> pair stream (all layers, spin means as dense rows)
//   for each one-electron layer l:
//       spin means g_up, g_dn of h^l                     (per walker)
//       P = [g_up | g_dn] V_g                             (matrix product)
//       X = [h_i | g_i_up | g_i_dn] V_h                   (matrix product)
//       h^{l+1} = tanh(X + P + b) (+ h^l)                 (forward Laplacian)
//   per spin: orbital head product, envelope x orbital (Eq. 4), slogdet
//   per walker: FP64 determinant sum, kinetic term (Eq. 3), Coulomb (Eq. 2)
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fn_internal.h"
#include "fn_kernels.h"

using namespace fn;

namespace {

thread_local std::string g_err;
int g_fp32_products = 0;     // bit 0 stream layers, bit 1 mean-field, bit 2 orbital head

fn_status fail(fn_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

// ---------------------------------------------------------------------------
// per-kernel timing (diagnostics)
// ---------------------------------------------------------------------------
enum KClass { K_STREAM_GEMM, K_WALKER_GEMM, K_HEAD_GEMM, K_FEATURES, K_PAIR, K_SPIN_MEAN, K_EPI, K_ENV, K_DET,
              K_COMBINE, K_PACK, K_PROPOSE, K_ACCEPT, K_BACKWARD, K_NCLASS };
const char *const kclass_names[K_NCLASS] = {"stream_gemm", "walker_gemm", "head_gemm", "features", "pair_stream",
                                           "spin_mean", "layer_epilogue", "envelope", "det", "combine", "pack",
                                           "propose", "accept", "backward"};
struct TimeRec { int cls; hipEvent_t a, b; };
std::mutex g_tmu;
bool g_timing = false;
thread_local bool g_no_alloc_call = false;   // the timing brackets create events: not inside such a call
int g_timing_only = -1;            // record one class only (-1: every class)
std::vector<TimeRec> g_recs;
std::vector<hipEvent_t> g_free_events;
double g_tot_ms[K_NCLASS];
int64_t g_tot_n[K_NCLASS];

hipEvent_t take_event()
{
    if (!g_free_events.empty()) {
        hipEvent_t e = g_free_events.back();
        g_free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// brackets the launches inside its lifetime when timing is enabled
struct Timed {
    int cls;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(int c, hipStream_t s) : cls(c), st(s)
    {
        if (!g_timing || g_no_alloc_call || (g_timing_only >= 0 && c != g_timing_only)) return;
        std::lock_guard<std::mutex> lk(g_tmu);
        a = take_event();
        if (a) (void)hipEventRecord(a, st);
    }
    ~Timed()
    {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_tmu);
        hipEvent_t b = take_event();
        if (!b) return;
        (void)hipEventRecord(b, st);
        g_recs.push_back({cls, a, b});
    }
};

void drain_timing()
{
    for (auto &r : g_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_tot_ms[r.cls] += ms;
            g_tot_n[r.cls] += 1;
        }
        g_free_events.push_back(r.a);
        g_free_events.push_back(r.b);
    }
    g_recs.clear();
}

struct Ctx {
    Sys s;
    ParamLayout P;
    Widths W;
    int prec;
    bool f64;
    size_t esz;      // bytes of the stream scalar (float or double)
    int smode;       // per-electron stream-layer products
    int wmode;       // per-walker mean-field products
    int hmode;       // orbital head product
    bool round_v;    // the layer weights V and head weights w are their BF16 roundings (FN_BF16W*_MIXED)
    double vnn;
};

fn_status make_ctx(const fn_config *cfg, Ctx &c)
{
    if (!cfg) return fail(FN_EINVAL, "cfg is NULL");
    if (cfg->n_nuc < 1 || cfg->n_nuc > FN_MAX_NUC) return fail(FN_EINVAL, "n_nuc out of range 1..32");
    if (!cfg->nuc_xyz || !cfg->nuc_z) return fail(FN_EINVAL, "nuc_xyz / nuc_z is NULL");
    if (cfg->n_up < 0 || cfg->n_down < 0 || cfg->n_up > FN_MAX_SPIN || cfg->n_down > FN_MAX_SPIN)
        return fail(FN_EINVAL, "n_up / n_down out of range 0..16");
    if (cfg->n_up + cfg->n_down < 1) return fail(FN_EINVAL, "no electrons");
    if (cfg->n_layers < 1 || cfg->n_layers > FN_MAX_LAYERS) return fail(FN_EINVAL, "n_layers out of range 1..8");
    if (cfg->w1 < 1 || cfg->w1 > FN_MAX_W1) return fail(FN_EINVAL, "w1 out of range 1..1024");
    if (cfg->w2 < 1 || cfg->w2 > FN_MAX_W2) return fail(FN_EINVAL, "w2 out of range 1..64");
    if (cfg->n_det < 1 || cfg->n_det > FN_MAX_DET) return fail(FN_EINVAL, "n_det out of range 1..32");
    if (cfg->precision < FN_FP64 || cfg->precision > FN_BF16W2_MIXED) return fail(FN_EINVAL, "unknown precision");
    if (cfg->envelope != FN_ENV_ANISOTROPIC && cfg->envelope != FN_ENV_ISOTROPIC)
        return fail(FN_EINVAL, "unknown envelope form");
    Sys &s = c.s;
    memset(&s, 0, sizeof(s));
    s.iso = cfg->envelope == FN_ENV_ISOTROPIC;
    s.M = cfg->n_nuc;
    s.nu = cfg->n_up;
    s.nd = cfg->n_down;
    s.N = s.nu + s.nd;
    s.L = cfg->n_layers;
    s.w1 = cfg->w1;
    s.w2 = cfg->w2;
    s.K = cfg->n_det;
    for (int m = 0; m < s.M; ++m) {
        for (int a = 0; a < 3; ++a) {
            s.R[m][a] = cfg->nuc_xyz[3 * m + a];
            if (!isfinite(s.R[m][a])) return fail(FN_EINVAL, "non-finite nucleus position");
        }
        s.Z[m] = cfg->nuc_z[m];
        if (!isfinite(s.Z[m])) return fail(FN_EINVAL, "non-finite nuclear charge");
    }
    c.P = make_layout(s);
    c.W = make_widths(s);
    c.prec = cfg->precision;
    c.f64 = c.prec == FN_FP64;
    c.esz = c.f64 ? 8 : 4;
    switch (c.prec) {
    case FN_FP64: c.smode = GEMM_F64; break;
    case FN_FP32: c.smode = GEMM_F32; break;
    case FN_BF16_MIXED: c.smode = GEMM_BF16; break;
    case FN_BF16X3_MIXED: c.smode = GEMM_BF16X3; break;
    case FN_BF16W_MIXED: c.smode = GEMM_BF16W3; break;
    case FN_BF16W2_MIXED: c.smode = GEMM_BF16W2; break;
    default: c.smode = GEMM_BF16X6; break;
    }
    // orbital head: FP32 operands; the six-product BF16 split carries them to
    // FP32 accuracy on the matrix cores, so the six-product mode uses it here
    // as well; in the BF16-weight modes the head weights are BF16 roundings
    // too, with the activations split as in the layers
    c.hmode = c.f64 ? GEMM_F64
                    : (c.smode == GEMM_BF16X6 ? GEMM_BF16X6
                                              : (c.smode == GEMM_BF16W3 || c.smode == GEMM_BF16W2 ? c.smode : GEMM_F32));
    c.wmode = c.smode;
    c.round_v = bf16_weight_mode(c.smode);
    // diagnostic: selected product classes on the FP32 matrix cores in the
    // split-BF16 modes (tuning switch "fp32_products")
    if (split_mode(c.smode)) {
        if (g_fp32_products & 1) c.smode = GEMM_F32;
        if (g_fp32_products & 2) c.wmode = GEMM_F32;
        if (g_fp32_products & 4) c.hmode = GEMM_F32;
    }
    double vnn = 0.0;
    for (int m = 0; m < s.M; ++m)
        for (int q = m + 1; q < s.M; ++q) {
            double d0 = s.R[m][0] - s.R[q][0], d1 = s.R[m][1] - s.R[q][1], d2 = s.R[m][2] - s.R[q][2];
            vnn += s.Z[m] * s.Z[q] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
    c.vnn = vnn;
    return FN_OK;
}

size_t gemm_elem(int mode) { return mode == GEMM_F64 ? 8 : (mode == GEMM_F32 ? 4 : 2); }

constexpr size_t ALIGN = 256;
size_t al(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of every buffer in the caller's workspace.
struct Plan {
    bool fl, save;
    int TR, rec;
    int64_t Bc;
    size_t wx[FN_MAX_LAYERS], wg[FN_MAX_LAYERS], wh[2], wb[2];
    size_t wx32[FN_MAX_LAYERS], wg32[FN_MAX_LAYERS];   // FP32 copies for the stacked kernel (0: none)
    size_t vr[FN_MAX_LAYERS];  // BF16-rounded layer weights V in the parameter layout (backward, BF16-weight modes)
    bool vround;
    bool stack32;
    size_t wpair;        // FP32 pair weights in the matrix-core pair kernel's layout (FP32 parameters only)
    int64_t wxpart[FN_MAX_LAYERS], wgpart[FN_MAX_LAYERS];   // elements per BF16 part
    size_t H[FN_MAX_LAYERS + 1], GI, G, Pw, X, O[2], Phi[2], DR, xp, lpn, u;
    // backward
    size_t Tl, GA[2], Ga[2], EP[2], Gy[2], Gz, SGz, Gh, Gg, GGI, PP, part, gacc, coeff, lsum;
    int64_t gi_layer_stride;   // elements
    int64_t npp, part_elems;
    size_t total;
};

constexpr size_t CHUNK_BYTES = (size_t)4 << 30;

fn_status make_plan(const Ctx &c, int64_t B, int op, Plan &p)
{
    const Sys &s = c.s;
    if (op < FN_OP_LOG_PSI || op > FN_OP_PARAM_GRAD) return fail(FN_EINVAL, "unknown op");
    p = Plan{};
    p.fl = op == FN_OP_LOCAL_ENERGY;
    p.save = op == FN_OP_PARAM_GRAD;
    const int n3 = 3 * s.N;
    p.TR = p.fl ? fl_rows(s.N) : 1;
    p.rec = n3 + 3;
    const int nmax = std::max(s.nu, s.nd);
    if (pair_stream_lds(s, p.fl, c.esz) > 64 * 1024) return fail(FN_EUNSUPPORTED, "pair stream exceeds LDS");
    if ((p.save ? det_lds(nmax, n3, false, sizeof(double)) : orbdet_lds(nmax, p.fl)) > 64 * 1024)
        return fail(FN_EUNSUPPORTED, "determinant exceeds LDS");
    if (p.save) {
        if (s.w1 % 32 != 0) return fail(FN_EUNSUPPORTED, "parameter gradients need w1 to be a multiple of 32");
        if (pair_backward_lds(s, c.esz) > 64 * 1024) return fail(FN_EUNSUPPORTED, "pair backward exceeds LDS");
        if (det_backward_lds(nmax) > 64 * 1024) return fail(FN_EUNSUPPORTED, "determinant backward exceeds LDS");
    }
    size_t o = 0;
    const size_t se = gemm_elem(c.smode), we = gemm_elem(c.wmode), he = gemm_elem(c.hmode), e = c.esz;
    const int np = weight_parts(c.smode), npw = weight_parts(c.wmode);
    for (int l = 0; l < s.L; ++l) {
        size_t nx = (size_t)s.w1 * (c.W.HWl[l] + c.W.GWl[l]), ng = (size_t)s.w1 * 2 * c.W.HWl[l];
        p.wxpart[l] = (int64_t)nx;
        p.wgpart[l] = (int64_t)ng;
        p.wx[l] = o; o = al(o + nx * se * np);
        p.wg[l] = o; o = al(o + ng * we * npw);
    }
    p.stack32 = p.fl && !p.save && c.wmode == c.smode && stack_fp32_weights(c.smode) &&
                stack_supported(c.smode, s.N, p.TR, s.w1, s.L);
    if (p.stack32)
        for (int l = 0; l < s.L; ++l) {
            p.wx32[l] = o; o = al(o + (size_t)p.wxpart[l] * sizeof(float));
            p.wg32[l] = o; o = al(o + (size_t)p.wgpart[l] * sizeof(float));
        }
    p.vround = p.save && c.round_v;
    if (p.vround)
        for (int l = 0; l < s.L; ++l) {
            p.vr[l] = o; o = al(o + (size_t)layer_din(s, l) * s.w1 * e);
        }
    p.wpair = o;
    if (c.esz == sizeof(float)) o = al(o + (size_t)pair_mfma_woff(s, s.L > 1 ? s.L - 1 : 0) * sizeof(float));
    for (int sp = 0; sp < 2; ++sp) {
        int n = sp == 0 ? s.nu : s.nd;
        size_t nh = (size_t)s.K * n * c.W.W1p;
        p.wh[sp] = o; o = al(o + nh * he * weight_parts(c.hmode));
        p.wb[sp] = o; if (p.save) o = al(o + (size_t)s.w1 * c.W.KNp[sp] * e);
    }
    // sizes that do not scale with the walker chunk
    p.npp = s.L > 1 ? (c.P.c2[s.L - 2] + s.w2 - c.P.W2[0]) : 0;
    int64_t pe = 0;
    if (p.save) {
        const int64_t kn_max = (int64_t)s.K * nmax;
        pe = std::max<int64_t>(pe, (int64_t)s.w1 * std::max<int64_t>(std::max(c.W.HWmax, 2 * c.W.GWmax), kn_max));
        pe = std::max<int64_t>(pe, kn_max * s.M * env_partials(s));
        pe = std::max<int64_t>(pe, p.npp);
        pe = std::max<int64_t>(pe, c.W.KNp[0] > c.W.KNp[1] ? c.W.KNp[0] : c.W.KNp[1]);
        pe *= max_splits();
    }
    p.part_elems = pe;
    p.part = o; o = al(o + (size_t)pe * e);
    const int64_t P = c.P.total;
    p.gacc = o; if (p.save) o = al(o + (size_t)P * 8);
    p.coeff = o; if (p.save) o = al(o + (size_t)B * 8);
    p.lsum = o; if (p.save) o = al(o + (size_t)2 * B * 8);
    p.xp = o; o = al(o + (size_t)B * n3 * 8);
    p.lpn = o; o = al(o + (size_t)B * 8);
    p.u = o; o = al(o + (size_t)B * 8);

    // per-walker buffers, laid out for a chunk of bc walkers
    const size_t TR = p.TR, N = s.N;
    const int nH = p.save ? s.L + 1 : 2;
    struct Item { size_t *off; size_t bytes_per_walker; };
    const size_t knp_max = std::max(c.W.KNp[0], c.W.KNp[1]);
    Item items[] = {
        {&p.GI, (size_t)s.L * N * TR * c.W.GWmax * e},
        {&p.G, TR * 2 * c.W.HWmax * e},
        {&p.Pw, TR * s.w1 * e},
        {&p.X, N * TR * s.w1 * e},
        {&p.O[0], (size_t)s.nu * TR * c.W.KNp[0] * e},
        {&p.O[1], (size_t)s.nd * TR * c.W.KNp[1] * e},
        {&p.Phi[0], p.save ? (size_t)s.K * TR * s.nu * s.nu * 8 : 0},   // stored for the backward only
        {&p.Phi[1], p.save ? (size_t)s.K * TR * s.nd * s.nd * 8 : 0},
        {&p.DR, (size_t)2 * s.K * p.rec * 8},
        {&p.Tl, p.save ? (size_t)s.L * N * s.w1 * e : 0},
        {&p.GA[0], p.save ? (size_t)s.K * s.nu * s.nu * 8 : 0},
        {&p.GA[1], p.save ? (size_t)s.K * s.nd * s.nd * 8 : 0},
        {&p.Ga[0], p.save ? (size_t)s.nu * c.W.KNp[0] * e : 0},
        {&p.Ga[1], p.save ? (size_t)s.nd * c.W.KNp[1] * e : 0},
        {&p.EP[0], p.save ? (size_t)s.K * s.nu * s.M * env_partials(s) * e : 0},
        {&p.EP[1], p.save ? (size_t)s.K * s.nd * s.M * env_partials(s) * e : 0},
        {&p.Gy[0], p.save ? N * s.w1 * e : 0},
        {&p.Gy[1], p.save ? N * s.w1 * e : 0},
        {&p.Gz, p.save ? N * s.w1 * e : 0},
        {&p.SGz, p.save ? (size_t)s.w1 * e : 0},
        {&p.Gh, p.save ? N * c.W.HWmax * e : 0},
        {&p.Gg, p.save ? 2 * c.W.HWmax * e : 0},
        {&p.GGI, p.save ? (size_t)s.L * N * c.W.GWmax * e : 0},
        {&p.PP, p.save ? N * (size_t)p.npp * e : 0},
    };
    (void)knp_max;
    size_t per_walker = N * TR * c.W.HWmax * e * nH;
    for (const Item &it : items) per_walker += it.bytes_per_walker;
    per_walker += sizeof(items) / sizeof(items[0]) * 8;   // alignment slack
    int64_t bc = (int64_t)(CHUNK_BYTES / std::max<size_t>(per_walker, 1));
    if (bc < 64) bc = 64;
    if (bc >= B) bc = B;
    else bc = bc / 64 * 64;
    if (bc < 1) bc = 1;
    p.Bc = bc;
    for (Item &it : items) {
        *it.off = o;
        o = al(o + it.bytes_per_walker * (size_t)bc);
    }
    // stream activations: nH buffers of one chunk each (2 ping-pong, or L + 1 kept for the backward pass)
    const size_t hbytes = al((size_t)bc * N * TR * c.W.HWmax * e);
    for (int l = 0; l < nH; ++l) {
        p.H[l] = o;
        o += hbytes;
    }
    p.gi_layer_stride = (int64_t)((size_t)bc * N * TR * c.W.GWmax);
    p.total = o;
    return FN_OK;
}

template <typename T>
void pack_weights(const Ctx &c, const Plan &p, const T *theta, char *ws, hipStream_t st)
{
    Timed t_(K_PACK, st);
    const Sys &s = c.s;
    PackList pl{};
    int64_t begin = 0;
    auto add = [&](const PackSeg &g) {
        pl.seg[pl.n] = g;
        pl.seg[pl.n].begin = begin;
        begin += g.count;
        ++pl.n;
    };
    for (int l = 0; l < s.L; ++l) {
        PackSeg g{};
        g.kind = 0; g.mode = c.smode; g.mode2 = c.wmode; g.off = c.P.V[l]; g.round = c.round_v;
        g.dh = layer_dh(s, l); g.dp = layer_dp(s, l); g.w1 = s.w1; g.HWl = c.W.HWl[l]; g.GWl = c.W.GWl[l];
        g.count = (int64_t)s.w1 * (g.HWl + g.GWl) + (int64_t)s.w1 * 2 * g.HWl;
        g.d0 = ws + p.wx[l]; g.d1 = ws + p.wg[l];
        add(g);
    }
    if (p.vround)
        for (int l = 0; l < s.L; ++l) {
            PackSeg g{};
            g.kind = 3; g.off = c.P.V[l]; g.count = (int64_t)layer_din(s, l) * s.w1;
            g.d0 = ws + p.vr[l];
            add(g);
        }
    if (p.stack32)
        for (int l = 0; l < s.L; ++l) {
            PackSeg g{};
            g.kind = 0; g.mode = GEMM_F32; g.mode2 = GEMM_F32; g.off = c.P.V[l]; g.round = c.round_v;
            g.dh = layer_dh(s, l); g.dp = layer_dp(s, l); g.w1 = s.w1; g.HWl = c.W.HWl[l]; g.GWl = c.W.GWl[l];
            g.count = (int64_t)s.w1 * (g.HWl + g.GWl) + (int64_t)s.w1 * 2 * g.HWl;
            g.d0 = ws + p.wx32[l]; g.d1 = ws + p.wg32[l];
            add(g);
        }
    for (int sp = 0; sp < 2; ++sp) {
        const int n = sp == 0 ? s.nu : s.nd;
        if (n == 0) continue;
        PackSeg g{};
        g.kind = 1; g.mode = c.hmode; g.off = c.P.w[sp]; g.round = c.round_v;
        g.w1 = s.w1; g.W1p = c.W.W1p; g.kn = s.K * n;
        g.count = (int64_t)g.kn * g.W1p;
        g.d0 = ws + p.wh[sp];
        add(g);
    }
    if (sizeof(T) == sizeof(float)) {
        const int wc = round_up(s.w2, 16);
        for (int l = 0; l + 1 < s.L; ++l) {
            PackSeg g{};
            g.kind = 2; g.mode = GEMM_F32; g.off = c.P.W2[l]; g.off2 = c.P.c2[l];
            g.dp = layer_dp(s, l); g.w2 = s.w2; g.wc = wc; g.ks = pair_mfma_kp(s, l) + 4;
            g.count = (int64_t)wc * g.ks + wc;
            g.d0 = ws + p.wpair + (size_t)pair_mfma_woff(s, l) * sizeof(float);
            add(g);
        }
    }
    launch_pack<T>(theta, pl, st);
    for (int sp = 0; sp < 2; ++sp) {
        const int n = sp == 0 ? s.nu : s.nd;
        if (n > 0 && p.save)
            launch_pack_head_bwd<T>(theta, c.P.w[sp], s.w1, s.K * n, c.W.KNp[sp], c.round_v, (T *)(ws + p.wb[sp]), st);
    }
}

// Forward pass of walkers [w0, w0 + b) (one chunk).  Weights are packed.  With
// p.save the stream activations of every layer and the tanh outputs are kept
// for the backward pass.
template <typename T>
void forward_chunk(const Ctx &c, const Plan &p, const T *theta, const double *xw, int64_t b, double *log_abs,
                   int8_t *sign, double *e_loc, double *parts, char *ws, hipStream_t st,
                   const AcceptArgs &acc = AcceptArgs{})
{
    const Sys &s = c.s;
    const int TR = p.TR, n3 = 3 * s.N;
    const bool fl = p.fl;
    auto Hbuf = [&](int l) -> T * { return (T *)(ws + p.H[p.save ? l : (l & 1)]); };
    T *GI = (T *)(ws + p.GI);
    T *G = (T *)(ws + p.G);
    T *Pw = (T *)(ws + p.Pw);
    T *X = (T *)(ws + p.X);
    double *DR = (double *)(ws + p.DR);
    const int64_t ldh = c.W.HWmax, ldg = c.W.GWmax;
    // every one-electron layer in one kernel with the activations in
    // registers: it forms the spin-mean products from the features itself
    bool regs = false;
    if constexpr (std::is_same<T, float>::value)
        regs = fl && !p.save && c.wmode == c.smode &&
               stack_regs_supported(c.smode, s.N, s.nu, TR, s.w1, s.L, c.W.HWl, c.W.GWl);
    // ... and the orbital head with it
    const bool head_fused = regs && stack_regs_head(c.smode, c.hmode, s.K, s.nu, s.nd, c.W.W1p);
    // the features and, in the same launch, the first layer's spin means
    // (not needed by the register kernel)
    {
        Timed t_(K_FEATURES, st);
        launch_features<T>(s, xw, b, TR, c.W.HWl[0], ldh, Hbuf(0), regs ? nullptr : G, st);
    }
    {
        Timed t_(K_PAIR, st);
        launch_pair_stream<T>(s, xw, theta, c.P, b, TR, fl, ldg, p.gi_layer_stride, c.W.GWl[0],
                              s.L > 1 ? c.W.GWl[1] : c.W.GWl[0],
                              sizeof(T) == sizeof(float) ? (const float *)(ws + p.wpair) : nullptr, GI, st);
    }
    bool g_ready = true;             // spin means of h^l already written (features, previous layer)
    bool stacked = false;
    if constexpr (std::is_same<T, float>::value) {
        // every one-electron layer in one kernel (activations in registers,
        // or in LDS)
        if (regs || (fl && !p.save && c.wmode == c.smode && stack_supported(c.smode, s.N, TR, s.w1, s.L))) {
            StackArgs sa{};
            sa.H0 = Hbuf(0); sa.ldh = ldh;
            sa.GI = GI; sa.ldgi = ldg; sa.gi_stride = p.gi_layer_stride;
            for (int l = 0; l < s.L; ++l) {
                sa.Wx[l] = (const uint16_t *)(ws + p.wx[l]); sa.wxpart[l] = p.wxpart[l];
                sa.Wg[l] = (const uint16_t *)(ws + p.wg[l]); sa.wgpart[l] = p.wgpart[l];
                if (p.stack32) {
                    sa.Wx32[l] = (const float *)(ws + p.wx32[l]);
                    sa.Wg32[l] = (const float *)(ws + p.wg32[l]);
                }
                sa.HW[l] = c.W.HWl[l]; sa.GW[l] = c.W.GWl[l];
                sa.bias[l] = theta + c.P.b[l];
            }
            sa.Hout = Hbuf(s.L);
            sa.B = b; sa.L = s.L; sa.nu = s.nu; sa.n3 = n3;
            if (regs && head_fused)
                for (int sp = 0; sp < 2; ++sp) {
                    sa.WH[sp] = (const uint16_t *)(ws + p.wh[sp]);
                    sa.O[sp] = (float *)(ws + p.O[sp]);
                    sa.ldo[sp] = c.W.KNp[sp];
                    sa.ldwh = c.W.W1p;
                }
            Timed t_(K_STREAM_GEMM, st);
            if (regs) launch_stack_regs(c.smode, sa, st);
            else launch_stack(c.smode, sa, s.N, st);
            stacked = true;
        }
    }
    for (int l = 0; l < s.L && !stacked; ++l) {
        const int dh = layer_dh(s, l), HWl = c.W.HWl[l], GWl = c.W.GWl[l];
        T *Hin = Hbuf(l), *Hout = Hbuf(l + 1);
        if (!g_ready) { Timed t_(K_SPIN_MEAN, st); launch_spin_mean<T>(Hin, ldh, b, s.N, s.nu, TR, dh, HWl, G, st); }
        g_ready = false;
        GemmArgs ga{};
        ga.A1 = G; ga.lda1 = 2 * HWl; ga.K1 = 2 * HWl;
        ga.W = ws + p.wg[l]; ga.wpart = p.wgpart[l]; ga.ldw = 2 * HWl;
        ga.C = Pw; ga.ldc = s.w1;
        // rows value .. Laplacian of each walker only: both epilogues read
        // no padding row of the per-walker part
        const int tr_live = fl ? n3 + 2 : TR;
        ga.rows = b * tr_live; ga.nout = s.w1;
        ga.rows_per_group = tr_live; ga.group_stride = TR;
        ga.c_rows_per_group = tr_live; ga.c_group_stride = TR;
        { Timed t_(K_WALKER_GEMM, st); (void)launch_gemm(c.wmode, ga, st); }
        bool fused = false;
        if constexpr (std::is_same<T, float>::value) fused = !p.save && stream_layer_supported(c.smode, TR, s.w1, c.W.W1p);
        if constexpr (std::is_same<T, float>::value) if (fused) {
            LayerArgs la{};
            la.A1 = Hin; la.lda1 = ldh; la.K1 = HWl;
            la.A2 = GI + (int64_t)l * p.gi_layer_stride; la.lda2 = ldg; la.K2 = GWl;
            la.W = ws + p.wx[l]; la.wpart = p.wxpart[l]; la.ldw = HWl + GWl; la.nout = s.w1;
            la.Pw = Pw; la.bias = theta + c.P.b[l];
            la.Hout = Hout; la.ldh_out = ldh;
            la.rows = b * s.N * TR; la.N = s.N; la.n3 = n3; la.w1 = s.w1; la.W1p = c.W.W1p;
            la.resid = l >= 1 ? 1 : 0;
            // the walker GEMM of layer l + 1 reads G before this kernel's
            // successor overwrites it, so G can take the next layer's means
            if (l + 1 < s.L && stream_layer_whole_walkers(s.N, TR) && c.W.HWl[l + 1] == c.W.W1p) {
                la.Gout = G;
                la.nu = s.nu;
                g_ready = true;
            }
            Timed t_(K_STREAM_GEMM, st);
            launch_stream_layer(c.smode, la, TR, st);
        }
        if (!fused) {
            GemmArgs gx{};
            gx.A1 = Hin; gx.lda1 = ldh; gx.K1 = HWl;
            gx.A2 = GI + (int64_t)l * p.gi_layer_stride; gx.lda2 = ldg; gx.K2 = GWl;
            gx.W = ws + p.wx[l]; gx.wpart = p.wxpart[l]; gx.ldw = HWl + GWl;
            gx.C = X; gx.ldc = s.w1;
            gx.nout = s.w1;
            const int tr_live = fl ? n3 + 2 : TR;
            if (8 * tr_live <= 7 * TR) {
                // live rows only: the epilogue reads no padding row of X
                gx.rows = b * s.N * tr_live;
                gx.rows_per_group = tr_live; gx.group_stride = TR;
                gx.c_rows_per_group = tr_live; gx.c_group_stride = TR;
            } else {
                gx.rows = b * s.N * TR; gx.rows_per_group = gx.rows;
            }
            { Timed t_(K_STREAM_GEMM, st); (void)launch_gemm(c.smode, gx, st); }
            Timed t_(K_EPI, st);
            T *Tout = p.save ? (T *)(ws + p.Tl) + (int64_t)l * b * s.N * s.w1 : nullptr;
            launch_layer_epi<T>(X, Pw, theta + c.P.b[l], Hin, Hout, ldh, b, s.N, TR, n3, s.w1, c.W.W1p,
                                l >= 1 ? 1 : 0, fl, Tout, st);
        }
    }
    T *HL = Hbuf(s.L);
    OrbSpins<T> orb{};
    // the orbital head of both spins (one launch when their tiles match)
    GemmArgs ghs[2]{};
    for (int sp = 0; sp < 2; ++sp) {
        const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
        if (n == 0) continue;
        T *O = (T *)(ws + p.O[sp]);
        GemmArgs &gh = ghs[sp];
        gh.A1 = HL; gh.lda1 = ldh; gh.K1 = c.W.W1p;
        gh.W = ws + p.wh[sp]; gh.ldw = c.W.W1p; gh.wpart = (int64_t)s.K * n * c.W.W1p;
        gh.C = O; gh.ldc = c.W.KNp[sp];
        gh.nout = s.K * n;
        gh.group_stride = (int64_t)s.N * TR; gh.row_offset = (int64_t)j0 * TR;
        const int tr_live = fl ? n3 + 2 : TR;
        if (8 * tr_live <= 7 * TR) {
            // rows value .. Laplacian of each electron only (the determinant
            // stage reads no padding row of O); not worth the broken tile
            // alignment when padding is under an eighth of the rows
            // (measured slower for 62 of 64)
            gh.rows = b * n * tr_live; gh.rows_per_group = (int64_t)n * tr_live;
            gh.rows_per_inner = tr_live; gh.inner_stride = TR;
            gh.c_rows_per_group = tr_live; gh.c_group_stride = TR;
        } else {
            gh.rows = b * n * TR; gh.rows_per_group = (int64_t)n * TR;
        }
    }
    if (!head_fused) {
        Timed t_(K_HEAD_GEMM, st);
        (void)launch_gemm2(c.hmode, ghs[0], ghs[1], st);
    }
    for (int sp = 0; sp < 2; ++sp) {
        const int n = sp == 0 ? s.nu : s.nd;
        if (n == 0) continue;
        T *O = (T *)(ws + p.O[sp]);
        if (fl || !p.save) {
            // orbital matrices formed and factorised in LDS or registers (both
            // spins in one launch below); only the backward needs them stored
            (sp ? orb.gof1 : orb.gof0) = c.P.g[sp];
            (sp ? orb.piof1 : orb.piof0) = c.P.pi[sp];
            (sp ? orb.sigof1 : orb.sigof0) = c.P.sig[sp];
            (sp ? orb.ldo1 : orb.ldo0) = c.W.KNp[sp];
            (sp ? orb.O1 : orb.O0) = O;
            continue;
        }
        double *Phi = (double *)(ws + p.Phi[sp]);
        {
            Timed t_(K_ENV, st);
            launch_envelope<T>(s, xw, theta, c.P.g[sp], c.P.pi[sp], c.P.sig[sp], sp, O, c.W.KNp[sp], b, TR, fl, Phi,
                               st);
        }
        { Timed t_(K_DET, st); launch_det(Phi, b, s.K, n, TR, n3, sp, fl, DR, p.rec, st); }
    }
    if (!fl && !p.save) {
        // value form with equal small spins: determinants and combine in one launch
        Timed t_(K_DET, st);
        if (launch_orbdet_combine<T>(s, xw, theta, orb, b, TR, log_abs, sign, acc, st)) return;
    }
    if (fl || !p.save) {
        Timed t_(K_DET, st);
        launch_orbdet<T>(s, xw, theta, orb, b, TR, fl, DR, p.rec, st);
    }
    Timed t_(K_COMBINE, st);
    launch_combine(s, xw, DR, p.rec, b, c.vnn, log_abs, sign, e_loc, parts, fl, acc, st);
}

// acc (value form only): Metropolis acceptance of the proposal x against
// acc's current walkers, folded into the combine kernel
template <typename T>
void forward(const Ctx &c, const Plan &p, const T *theta, const double *x, int64_t B, double *log_abs, int8_t *sign,
             double *e_loc, double *parts, char *ws, hipStream_t st, const AcceptArgs &acc = AcceptArgs{})
{
    const int n3 = 3 * c.s.N;
    for (int64_t w0 = 0; w0 < B; w0 += p.Bc) {
        const int64_t b = std::min(p.Bc, B - w0);
        AcceptArgs ac{};
        if (acc.x)
            ac = AcceptArgs{acc.x + w0 * n3, acc.xp + w0 * n3, acc.u + w0, acc.log_abs + w0,
                            acc.n_accept ? acc.n_accept + w0 : nullptr};
        forward_chunk<T>(c, p, theta, x + w0 * n3, b, log_abs ? log_abs + w0 : nullptr, sign ? sign + w0 : nullptr,
                         e_loc ? e_loc + w0 : nullptr, parts ? parts + 4 * w0 : nullptr, ws, st, ac);
    }
}

// Reverse pass for walkers [w0, w0 + b) after forward_chunk with p.save:
// accumulates sum_p coeff_p d log|psi_p| / d theta into the FP64 buffer gacc.
// With targets (Eq. 5 pretraining): the adjoint of the orbital matrices is
// scale (Phi - target) instead of the determinants' adjoint, and each
// walker's sum of squared differences goes to lsum[spin][walker].
struct PretrainTargets {
    const double *t[2];      // [B][K][n_s][n_s] of the whole batch, at this chunk's first walker
    double scale;            // 2 / B_total
    double *lsum[2];         // [B] of this chunk
};

template <typename T>
void backward_chunk(const Ctx &c, const Plan &p, const T *theta, const double *xw, const double *coeff, int64_t b,
                    char *ws, hipStream_t st, const PretrainTargets *pre = nullptr)
{
    Timed t_(K_BACKWARD, st);
    const Sys &s = c.s;
    const int N = s.N, w1 = s.w1;
    const int gmode = c.f64 ? GEMM_F64 : GEMM_F32;
    double *gacc = (double *)(ws + p.gacc);
    T *part = (T *)(ws + p.part);
    const int64_t rows = b * N;
    const int64_t ldh = c.W.HWmax, ldg = c.W.GWmax;
    T *Gy = (T *)(ws + p.Gy[0]), *Gy2 = (T *)(ws + p.Gy[1]);
    // determinants, envelope and orbital head, per spin
    for (int sp = 0; sp < 2; ++sp) {
        const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
        if (n == 0) continue;
        const int kn = s.K * n, KNp = c.W.KNp[sp];
        double *GA = (double *)(ws + p.GA[sp]);
        T *Ga = (T *)(ws + p.Ga[sp]);
        T *EP = (T *)(ws + p.EP[sp]);
        if (pre)
            launch_pretrain_adjoint((const double *)(ws + p.Phi[sp]), pre->t[sp], b, s.K, n, pre->scale, GA,
                                    pre->lsum[sp], st);
        else
            launch_det_backward((const double *)(ws + p.Phi[sp]), (const double *)(ws + p.DR), coeff, b, s.K, n, sp,
                                s.nu, s.nd, p.rec, GA, st);
        launch_env_backward<T>(s, xw, theta, c.P.g[sp], c.P.pi[sp], c.P.sig[sp], sp, (const T *)(ws + p.O[sp]), KNp,
                               GA, b, KNp, Ga, EP, st);
        launch_colsum<T>(EP, (int64_t)kn * s.M * env_partials(s), kn * s.M * env_partials(s), b, part, gacc, c.P.pi[sp],
                         env_partials(s), c.P.sig[sp], st);
        launch_colsum<T>(Ga, KNp, kn, b * n, part, gacc, c.P.g[sp], 0, 0, st);
        launch_tn<T>((const T *)(ws + p.H[s.L]), ldh, w1, Ga, KNp, kn, b * n, n, N, j0, part, gacc, c.P.w[sp], kn, st);
        GemmArgs g{};
        g.A1 = Ga; g.lda1 = KNp; g.K1 = KNp;
        g.W = ws + p.wb[sp]; g.ldw = KNp;
        g.C = Gy; g.ldc = w1;
        g.rows = b * n; g.nout = w1;
        g.rows_per_group = g.rows;
        g.c_rows_per_group = n; g.c_group_stride = N; g.c_row_offset = j0;
        (void)launch_gemm(gmode, g, st);
    }
    // one-electron layers, top down
    T *Gz = (T *)(ws + p.Gz), *SGz = (T *)(ws + p.SGz), *Gh = (T *)(ws + p.Gh), *Gg = (T *)(ws + p.Gg);
    T *G = (T *)(ws + p.G);
    T *GGI = (T *)(ws + p.GGI);
    for (int l = s.L - 1; l >= 0; --l) {
        const int dh = layer_dh(s, l), dp = layer_dp(s, l), HWl = c.W.HWl[l];
        const T *Hl = (const T *)(ws + p.H[l]);
        const T *Tl = (const T *)(ws + p.Tl) + (int64_t)l * rows * w1;
        const int64_t voff = c.P.V[l];
        // the layer's weights as the forward multiplied with them
        const T *Vl = p.vround ? (const T *)(ws + p.vr[l]) : theta + voff;
        launch_bwd_gz<T>(Gy, Tl, b, N, w1, Gz, SGz, st);
        launch_colsum<T>(Gz, w1, w1, rows, part, gacc, c.P.b[l], 0, 0, st);
        launch_tn<T>(Hl, ldh, dh, Gz, w1, w1, rows, 0, 0, 0, part, gacc, voff, w1, st);
        const T *GIl = (const T *)(ws + p.GI) + (int64_t)l * p.gi_layer_stride;
        launch_tn<T>(GIl, ldg, 2 * dp, Gz, w1, w1, rows, 0, 0, 0, part, gacc, voff + (int64_t)3 * dh * w1, w1, st);
        launch_spin_mean<T>(Hl, ldh, b, N, s.nu, 1, dh, HWl, G, st);
        launch_tn<T>(G, 2 * HWl, dh, SGz, w1, w1, b, 0, 0, 0, part, gacc, voff + (int64_t)dh * w1, w1, st);
        launch_tn<T>(G + HWl, 2 * HWl, dh, SGz, w1, w1, b, 0, 0, 0, part, gacc, voff + (int64_t)2 * dh * w1, w1, st);
        // adjoints of the pair means (to the pair stream) and of h^l
        GemmArgs gq{};
        gq.A1 = Gz; gq.lda1 = w1; gq.K1 = w1;
        gq.W = Vl + (int64_t)3 * dh * w1; gq.ldw = w1;
        gq.C = GGI + (int64_t)l * p.gi_layer_stride; gq.ldc = ldg;
        gq.rows = rows; gq.nout = 2 * dp;
        gq.rows_per_group = rows;
        (void)launch_gemm(gmode, gq, st);
        if (l == 0) break;
        GemmArgs gh{};
        gh.A1 = Gz; gh.lda1 = w1; gh.K1 = w1;
        gh.W = Vl; gh.ldw = w1;
        gh.C = Gh; gh.ldc = dh;
        gh.rows = rows; gh.nout = dh;
        gh.rows_per_group = rows;
        (void)launch_gemm(gmode, gh, st);
        GemmArgs gg{};
        gg.A1 = SGz; gg.lda1 = w1; gg.K1 = w1;
        gg.W = Vl + (int64_t)dh * w1; gg.ldw = w1;
        gg.C = Gg; gg.ldc = 2 * dh;
        gg.rows = b; gg.nout = 2 * dh;
        gg.rows_per_group = b;
        (void)launch_gemm(gmode, gg, st);
        launch_bwd_gh<T>(Gh, Gy, Gg, b, N, s.nu, dh, w1, 1, Gy2, st);
        std::swap(Gy, Gy2);
    }
    if (s.L > 1) {
        T *PP = (T *)(ws + p.PP);
        // one PP row per pair-backward workgroup
        const int64_t npr = launch_pair_backward<T>(s, xw, theta, c.P, b, GGI, ldg, p.gi_layer_stride,
                                                    sizeof(T) == sizeof(float) ? (const float *)(ws + p.wpair) : nullptr,
                                                    PP, p.npp, st);
        launch_colsum<T>(PP, p.npp, (int)p.npp, npr, part, gacc, c.P.W2[0], 0, 0, st);
    }
}

fn_status check_ws(const Plan &p, void *ws, size_t ws_bytes)
{
    if (!ws) return fail(FN_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % ALIGN) return fail(FN_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < p.total)
        return fail(FN_ENOMEM, "workspace too small: need " + std::to_string(p.total) + " bytes, got " +
                                   std::to_string(ws_bytes));
    return FN_OK;
}

fn_status hip_status()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FN_EHIP, std::string("HIP error: ") + hipGetErrorString(e));
    return FN_OK;
}

template <typename T>
fn_status run_forward(const Ctx &c, const Plan &p, const void *theta, const double *x, int64_t B, double *log_abs,
                      int8_t *sign, double *e_loc, double *parts, void *ws, hipStream_t st)
{
    pack_weights<T>(c, p, (const T *)theta, (char *)ws, st);
    forward<T>(c, p, (const T *)theta, x, B, log_abs, sign, e_loc, parts, (char *)ws, st);
    return hip_status();
}

template <typename T>
fn_status run_metropolis(const Ctx &c, const Plan &p, const void *theta, double *x, double *log_abs, int64_t B,
                         int32_t n_steps, double sigma, uint64_t seed, uint64_t step0, uint32_t stream_id,
                         const double *z, const double *u, int32_t *n_accept, void *ws, hipStream_t st)
{
    char *w = (char *)ws;
    const int n3 = 3 * c.s.N;
    pack_weights<T>(c, p, (const T *)theta, w, st);
    double *xp = (double *)(w + p.xp), *lpn = (double *)(w + p.lpn), *uu = (double *)(w + p.u);
    for (int32_t k = 0; k < n_steps; ++k) {
        {
            Timed t_(K_PROPOSE, st);
            launch_propose(x, B, n3, sigma, seed, step0 + (uint64_t)k, stream_id,
                           z ? z + (int64_t)k * B * n3 : nullptr, u ? u + (int64_t)k * B : nullptr, xp, uu, st);
        }
        // the acceptance runs in the combine kernel of the proposal's value pass
        forward<T>(c, p, (const T *)theta, xp, B, lpn, nullptr, nullptr, nullptr, w, st,
                   AcceptArgs{x, xp, uu, log_abs, n_accept});
    }
    return hip_status();
}

// grouped moves: every job advances n_steps together; job q's step counter
// at move k is its step0 + k
template <typename T>
fn_status run_metropolis_group(const Ctx &c, const Plan &p, const void *theta, double *x, double *log_abs, int64_t B,
                               int32_t n_steps, double sigma, const fn_group_job *jobs, int32_t n_jobs,
                               int32_t *n_accept, void *ws, hipStream_t st)
{
    char *w = (char *)ws;
    const int n3 = 3 * c.s.N;
    pack_weights<T>(c, p, (const T *)theta, w, st);
    double *xp = (double *)(w + p.xp), *lpn = (double *)(w + p.lpn), *uu = (double *)(w + p.u);
    GroupTable g{};
    g.n = n_jobs;
    for (int q = 0; q < n_jobs; ++q) {
        g.w0[q] = jobs[q].walker0;
        g.k0[q] = (uint32_t)jobs[q].seed;
        g.k1[q] = (uint32_t)(jobs[q].seed >> 32);
        g.stream[q] = jobs[q].stream_id;
    }
    g.w0[n_jobs] = B;
    for (int32_t k = 0; k < n_steps; ++k) {
        for (int q = 0; q < n_jobs; ++q) g.step[q] = (uint32_t)(jobs[q].step0 + (uint64_t)k);
        {
            Timed t_(K_PROPOSE, st);
            launch_propose_group(x, B, n3, sigma, g, xp, uu, st);
        }
        forward<T>(c, p, (const T *)theta, xp, B, lpn, nullptr, nullptr, nullptr, w, st,
                   AcceptArgs{x, xp, uu, log_abs, n_accept});
    }
    return hip_status();
}

template <typename T>
fn_status run_pretrain(const Ctx &c, const Plan &p, const void *theta, const double *x, int64_t B,
                       const double *target_up, const double *target_dn, double *loss, void *grad, void *ws,
                       hipStream_t st)
{
    char *w = (char *)ws;
    const T *th = (const T *)theta;
    const int n3 = 3 * c.s.N;
    double *gacc = (double *)(w + p.gacc);
    double *lsum = (double *)(w + p.lsum);
    launch_zero_f64(gacc, c.P.total, st);
    launch_zero_f64(lsum, 2 * B, st);
    pack_weights<T>(c, p, th, w, st);
    double *lp = (double *)(w + p.lpn);
    const int64_t per[2] = {(int64_t)c.s.K * c.s.nu * c.s.nu, (int64_t)c.s.K * c.s.nd * c.s.nd};
    for (int64_t w0 = 0; w0 < B; w0 += p.Bc) {
        const int64_t b = std::min(p.Bc, B - w0);
        forward_chunk<T>(c, p, th, x + w0 * n3, b, lp + w0, nullptr, nullptr, nullptr, w, st);
        PretrainTargets pre{};
        pre.t[0] = c.s.nu ? target_up + w0 * per[0] : nullptr;
        pre.t[1] = c.s.nd ? target_dn + w0 * per[1] : nullptr;
        pre.scale = 2.0 / (double)B;
        pre.lsum[0] = lsum + w0;
        pre.lsum[1] = lsum + B + w0;
        backward_chunk<T>(c, p, th, x + w0 * n3, nullptr, b, w, st, &pre);
    }
    launch_grad_out<T>(gacc, c.P.total, (T *)grad, st);
    if (loss) launch_pretrain_loss(lsum, B, loss, st);
    return hip_status();
}

template <typename T>
fn_status run_backward(const Ctx &c, const Plan &p, const void *theta, const double *x, int64_t B,
                       const double *coeff_in, const double *e_loc, double *stats, void *grad, void *ws, hipStream_t st)
{
    char *w = (char *)ws;
    const T *th = (const T *)theta;
    const int n3 = 3 * c.s.N;
    double *gacc = (double *)(w + p.gacc);
    const double *coeff = coeff_in;
    if (e_loc) {
        double *cf = (double *)(w + p.coeff);
        launch_energy_stats(e_loc, B, stats, cf, st);
        coeff = cf;
    }
    launch_zero_f64(gacc, c.P.total, st);
    pack_weights<T>(c, p, th, w, st);
    double *lp = (double *)(w + p.lpn);
    for (int64_t w0 = 0; w0 < B; w0 += p.Bc) {
        const int64_t b = std::min(p.Bc, B - w0);
        forward_chunk<T>(c, p, th, x + w0 * n3, b, lp + w0, nullptr, nullptr, nullptr, w, st);
        backward_chunk<T>(c, p, th, x + w0 * n3, coeff + w0, b, w, st);
    }
    launch_grad_out<T>(gacc, c.P.total, (T *)grad, st);
    return hip_status();
}

}  // namespace

fn_status fn::api_fail(fn_status st, const char *msg) { return fail(st, msg); }

extern "C" {

int64_t fn_param_count(const fn_config *cfg)
{
    Ctx c;
    if (make_ctx(cfg, c) != FN_OK) return -1;
    return c.P.total;
}

size_t fn_workspace_bytes(const fn_config *cfg, int64_t B, int32_t op)
{
    Ctx c;
    if (make_ctx(cfg, c) != FN_OK) return 0;
    if (B < 0) { fail(FN_EINVAL, "B < 0"); return 0; }
    Plan p;
    if (make_plan(c, B, op, p) != FN_OK) return 0;
    return p.total;
}

fn_status fn_log_psi(const fn_config *cfg, const void *theta, const double *x, int64_t B, double *log_abs_psi,
                     int8_t *sign, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (B < 0) return fail(FN_EINVAL, "B < 0");
    if (B == 0) return FN_OK;
    if (!theta || !x || !log_abs_psi) return fail(FN_EINVAL, "theta, x or log_abs_psi is NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    Plan p;
    if ((r = make_plan(c, B, FN_OP_LOG_PSI, p))) return r;
    if ((r = check_ws(p, ws, ws_bytes))) return r;
    hipStream_t st = (hipStream_t)stream;
    return c.f64 ? run_forward<double>(c, p, theta, x, B, log_abs_psi, sign, nullptr, nullptr, ws, st)
                 : run_forward<float>(c, p, theta, x, B, log_abs_psi, sign, nullptr, nullptr, ws, st);
}

fn_status fn_local_energy(const fn_config *cfg, const void *theta, const double *x, int64_t B, double *e_loc,
                          double *log_abs_psi, double *parts, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (B < 0) return fail(FN_EINVAL, "B < 0");
    if (B == 0) return FN_OK;
    if (!theta || !x || !e_loc) return fail(FN_EINVAL, "theta, x or e_loc is NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    Plan p;
    if ((r = make_plan(c, B, FN_OP_LOCAL_ENERGY, p))) return r;
    if ((r = check_ws(p, ws, ws_bytes))) return r;
    hipStream_t st = (hipStream_t)stream;
    return c.f64 ? run_forward<double>(c, p, theta, x, B, log_abs_psi, nullptr, e_loc, parts, ws, st)
                 : run_forward<float>(c, p, theta, x, B, log_abs_psi, nullptr, e_loc, parts, ws, st);
}

static fn_status metropolis_common(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi, int64_t B,
                                   int32_t n_steps, double sigma, uint64_t seed, uint64_t step0, uint32_t stream_id,
                                   const double *z, const double *u, int32_t *n_accept, void *ws, size_t ws_bytes,
                                   void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (B < 0) return fail(FN_EINVAL, "B < 0");
    if (n_steps < 0) return fail(FN_EINVAL, "n_steps < 0");
    if (!(sigma >= 0.0) || !isfinite(sigma)) return fail(FN_EINVAL, "sigma must be finite and >= 0");
    if (B == 0 || n_steps == 0) return FN_OK;
    if (!theta || !x || !log_abs_psi) return fail(FN_EINVAL, "theta, x or log_abs_psi is NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    Plan p;
    if ((r = make_plan(c, B, FN_OP_METROPOLIS, p))) return r;
    if ((r = check_ws(p, ws, ws_bytes))) return r;
    hipStream_t st = (hipStream_t)stream;
    return c.f64 ? run_metropolis<double>(c, p, theta, x, log_abs_psi, B, n_steps, sigma, seed, step0, stream_id, z, u,
                                          n_accept, ws, st)
                 : run_metropolis<float>(c, p, theta, x, log_abs_psi, B, n_steps, sigma, seed, step0, stream_id, z, u,
                                         n_accept, ws, st);
}

fn_status vmc_metropolis_step(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi, int64_t B,
                              int32_t n_steps, double sigma, uint64_t seed, uint64_t step0, uint32_t stream_id,
                              int32_t *n_accept, void *ws, size_t ws_bytes, void *stream)
{
    return metropolis_common(cfg, theta, x, log_abs_psi, B, n_steps, sigma, seed, step0, stream_id, nullptr, nullptr,
                             n_accept, ws, ws_bytes, stream);
}

fn_status vmc_metropolis_step_ext(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi, int64_t B,
                                  int32_t n_steps, double sigma, const double *z, const double *u, int32_t *n_accept,
                                  void *ws, size_t ws_bytes, void *stream)
{
    if (!z || !u) return fail(FN_EINVAL, "z or u is NULL");
    return metropolis_common(cfg, theta, x, log_abs_psi, B, n_steps, sigma, 0, 0, 0, z, u, n_accept, ws, ws_bytes,
                             stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Workspace of vmc_metropolis_step_noalloc: a fixed device array, one copy per
// GPU, held until the process ends.  Host code uses the per-device address
// from hipGetSymbolAddress, never the array's name.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// the address of the current device's copy (looked up once per device)
fn_status scratch_for_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FN_EHIP, "hipGetDevice failed");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(FN_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FN_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FN_OK;
}

}  // namespace

extern "C" {

fn_status vmc_metropolis_step_noalloc(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi,
                                      int64_t B, int32_t n_steps, double sigma, uint64_t seed, uint64_t step0,
                                      uint32_t stream_id, int32_t *n_accept, void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (B < 0) return fail(FN_EINVAL, "B < 0");
    if (n_steps < 0) return fail(FN_EINVAL, "n_steps < 0");
    if (!(sigma >= 0.0) || !isfinite(sigma)) return fail(FN_EINVAL, "sigma must be finite and >= 0");
    if (B == 0 || n_steps == 0) return FN_OK;
    if (!theta || !x || !log_abs_psi) return fail(FN_EINVAL, "theta, x or log_abs_psi is NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    Plan p;
    if ((r = make_plan(c, B, FN_OP_METROPOLIS, p))) return r;
    if (p.total > NOALLOC_SCRATCH_BYTES)
        return fail(FN_ENOMEM, "needs " + std::to_string(p.total) + " bytes of scratch; the fixed scratch holds " +
                                   std::to_string(NOALLOC_SCRATCH_BYTES) + " (use vmc_metropolis_step with a workspace)");
    void *ws = nullptr;
    if ((r = scratch_for_current_device(&ws))) return r;
    struct NoAlloc {
        NoAlloc() { g_no_alloc_call = true; }
        ~NoAlloc() { g_no_alloc_call = false; }
    } no_alloc_;
    hipStream_t st = (hipStream_t)stream;
    return c.f64 ? run_metropolis<double>(c, p, theta, x, log_abs_psi, B, n_steps, sigma, seed, step0, stream_id,
                                          nullptr, nullptr, n_accept, ws, st)
                 : run_metropolis<float>(c, p, theta, x, log_abs_psi, B, n_steps, sigma, seed, step0, stream_id,
                                         nullptr, nullptr, n_accept, ws, st);
}

fn_status vmc_metropolis_step_group(const fn_config *cfg, const void *theta, const fn_group_job *jobs, int32_t n_jobs,
                                    double *x, double *log_abs_psi, int32_t *n_accept, int64_t B_total,
                                    int32_t n_steps, double sigma, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (!jobs || n_jobs < 1 || n_jobs > FN_MAX_GROUP_JOBS) return fail(FN_EINVAL, "n_jobs out of range 1..64");
    if (B_total < 1) return fail(FN_EINVAL, "B_total < 1");
    int64_t next = 0;
    for (int q = 0; q < n_jobs; ++q) {
        if (jobs[q].B < 1) return fail(FN_EINVAL, "a job has no walkers");
        if (jobs[q].walker0 != next) return fail(FN_EINVAL, "jobs must tile the walkers in order without gaps");
        next += jobs[q].B;
    }
    if (next != B_total) return fail(FN_EINVAL, "the jobs' walkers do not add up to B_total");
    if (n_steps < 0) return fail(FN_EINVAL, "n_steps < 0");
    if (!(sigma >= 0.0) || !isfinite(sigma)) return fail(FN_EINVAL, "sigma must be finite and >= 0");
    if (n_steps == 0) return FN_OK;
    if (!theta || !x || !log_abs_psi) return fail(FN_EINVAL, "theta, x or log_abs_psi is NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    Plan p;
    if ((r = make_plan(c, B_total, FN_OP_METROPOLIS, p))) return r;
    if ((r = check_ws(p, ws, ws_bytes))) return r;
    struct Suppress {
        bool prev = g_splitk_suppressed;
        Suppress() { g_splitk_suppressed = true; }
        ~Suppress() { g_splitk_suppressed = prev; }
    } suppress_;
    hipStream_t st = (hipStream_t)stream;
    return c.f64 ? run_metropolis_group<double>(c, p, theta, x, log_abs_psi, B_total, n_steps, sigma, jobs, n_jobs,
                                                n_accept, ws, st)
                 : run_metropolis_group<float>(c, p, theta, x, log_abs_psi, B_total, n_steps, sigma, jobs, n_jobs,
                                               n_accept, ws, st);
}

static fn_status grad_common(const fn_config *cfg, const void *theta, const double *x, int64_t B,
                             const double *coeff, const double *e_loc, double *stats, void *grad, void *ws,
                             size_t ws_bytes, void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (B < 0) return fail(FN_EINVAL, "B < 0");
    if (!grad || !theta) return fail(FN_EINVAL, "theta or grad is NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    if (B > 0 && !x) return fail(FN_EINVAL, "x is NULL");
    Plan p;
    if ((r = make_plan(c, B, FN_OP_PARAM_GRAD, p))) return r;
    if ((r = check_ws(p, ws, ws_bytes))) return r;
    hipStream_t st = (hipStream_t)stream;
    if (B == 0) {
        launch_zero_f64((double *)((char *)ws + p.gacc), c.P.total, st);
        if (c.f64) launch_grad_out<double>((double *)((char *)ws + p.gacc), c.P.total, (double *)grad, st);
        else launch_grad_out<float>((double *)((char *)ws + p.gacc), c.P.total, (float *)grad, st);
        return hip_status();
    }
    return c.f64 ? run_backward<double>(c, p, theta, x, B, coeff, e_loc, stats, grad, ws, st)
                 : run_backward<float>(c, p, theta, x, B, coeff, e_loc, stats, grad, ws, st);
}

fn_status fn_pretrain_grad(const fn_config *cfg, const void *theta, const double *x, int64_t B, const double *target_up,
                           const double *target_dn, double *loss, void *grad, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    fn_status r = make_ctx(cfg, c);
    if (r) return r;
    if (B < 1) return fail(FN_EINVAL, "B < 1");
    if (!theta || !x || !grad) return fail(FN_EINVAL, "theta, x or grad is NULL");
    if ((c.s.nu && !target_up) || (c.s.nd && !target_dn)) return fail(FN_EINVAL, "a spin's targets are NULL");
    if (((uintptr_t)theta) % 16) return fail(FN_EINVAL, "theta must be 16-byte aligned");
    Plan p;
    if ((r = make_plan(c, B, FN_OP_PARAM_GRAD, p))) return r;
    if ((r = check_ws(p, ws, ws_bytes))) return r;
    hipStream_t st = (hipStream_t)stream;
    return c.f64 ? run_pretrain<double>(c, p, theta, x, B, target_up, target_dn, loss, grad, ws, st)
                 : run_pretrain<float>(c, p, theta, x, B, target_up, target_dn, loss, grad, ws, st);
}

fn_status fn_param_grad(const fn_config *cfg, const void *theta, const double *x, int64_t B, const double *e_loc,
                        void *grad, double *stats, void *ws, size_t ws_bytes, void *stream)
{
    if (B > 0 && !e_loc) return fail(FN_EINVAL, "e_loc is NULL");
    return grad_common(cfg, theta, x, B, nullptr, e_loc, stats, grad, ws, ws_bytes, stream);
}

fn_status fn_log_psi_vjp(const fn_config *cfg, const void *theta, const double *x, int64_t B, const double *coeff,
                         void *grad, void *ws, size_t ws_bytes, void *stream)
{
    if (B > 0 && !coeff) return fail(FN_EINVAL, "coeff is NULL");
    return grad_common(cfg, theta, x, B, coeff, nullptr, nullptr, grad, ws, ws_bytes, stream);
}

fn_status fn_energy_stats(const double *e_loc, int64_t B, double *stats, double *coeff, void *stream)
{
    if (B < 1) return fail(FN_EINVAL, "B < 1");
    if (!e_loc) return fail(FN_EINVAL, "e_loc is NULL");
    if (!stats && !coeff) return fail(FN_EINVAL, "stats and coeff are both NULL");
    launch_energy_stats(e_loc, B, stats, coeff, (hipStream_t)stream);
    return hip_status();
}

const char *fn_last_error(void) { return g_err.c_str(); }

fn_status fn_tuning_set(const char *name, int64_t value)
{
    if (!name) return fail(FN_EINVAL, "NULL name");
    if (strcmp(name, "fused_layer") == 0) {
        fn::g_use_fused_layer = value != 0;
        return FN_OK;
    }
    if (strcmp(name, "gemm_splitk") == 0) {
        fn::g_gemm_splitk = value != 0;
        return FN_OK;
    }
    if (strcmp(name, "gemm_wide") == 0) {
        fn::g_gemm_wide = value != 0;
        return FN_OK;
    }
    if (strcmp(name, "layer_dma") == 0) {
        fn::g_layer_dma = value != 0;
        return FN_OK;
    }
    if (strcmp(name, "pair_mfma") == 0) {
        fn::g_pair_mfma = value != 0;
        return FN_OK;
    }
    if (strcmp(name, "pair_oc") == 0) {
        if (value != 0 && value != 1 && value != 2 && value != 4) return fail(FN_EINVAL, "pair_oc: 0, 1, 2 or 4");
        fn::g_pair_oc = (int)value;
        return FN_OK;
    }
    if (strcmp(name, "stack_regs") == 0) {
        if (value < 0 || value > 1) return fail(FN_EINVAL, "stack_regs: 0 or 1");
        fn::g_stack_regs = value != 0;
        return FN_OK;
    }
    if (strcmp(name, "layer_stack") == 0) {
        if (value < 0 || value > 2) return fail(FN_EINVAL, "layer_stack: 0, 1 or 2");
        fn::g_use_stack = (int)value;
        return FN_OK;
    }
    if (strcmp(name, "stack_shape") == 0) {
        if (value < 0 || value > 2) return fail(FN_EINVAL, "stack_shape: 0, 1 or 2");
        fn::g_stack_shape = (int)value;
        return FN_OK;
    }
    if (strcmp(name, "fp32_products") == 0) {
        if (value < 0 || value > 7) return fail(FN_EINVAL, "fp32_products: 0..7");
        g_fp32_products = (int)value;
        return FN_OK;
    }
    if (strcmp(name, "det_stage") == 0) {
        if (value < 0 || value > 1) return fail(FN_EINVAL, "det_stage: 0 or 1");
        fn::g_det_stage = (int)value;
        return FN_OK;
    }
    if (strcmp(name, "pair_items") == 0) {
        if (value < 0 || value > 4096) return fail(FN_EINVAL, "pair_items: 0..4096");
        fn::g_pair_items = (int)value;
        return FN_OK;
    }
    return fail(FN_EINVAL, std::string("unknown tuning switch ") + name);
}

fn_status fn_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return FN_OK;
}

fn_status fn_timing_select(const char *name)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!name) {
        g_timing_only = -1;
        return FN_OK;
    }
    for (int k = 0; k < K_NCLASS; ++k)
        if (strcmp(name, kclass_names[k]) == 0) {
            g_timing_only = k;
            return FN_OK;
        }
    return fail(FN_EINVAL, std::string("unknown kernel class ") + name);
}

fn_status fn_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    drain_timing();
    for (int k = 0; k < K_NCLASS; ++k) { g_tot_ms[k] = 0.0; g_tot_n[k] = 0; }
    return FN_OK;
}

fn_status fn_timing_read(const char *name, double *total_ms, int64_t *launches)
{
    if (!name || !total_ms || !launches) return fail(FN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    drain_timing();
    for (int k = 0; k < K_NCLASS; ++k)
        if (strcmp(name, kclass_names[k]) == 0) {
            *total_ms = g_tot_ms[k];
            *launches = g_tot_n[k];
            return FN_OK;
        }
    return fail(FN_EINVAL, std::string("unknown kernel class ") + name);
}

}  // extern "C"
