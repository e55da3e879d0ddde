// fn_net.hip -- element-wise and per-walker kernels of the FermiNet forward
// pass with a forward-mode Laplacian (FermiNet Model section of the paper;
// the kinetic term of Eq. 3 needs the gradient and Laplacian of log|psi|
// with respect to all 3N electron coordinates).
//
// Every quantity q carries rows (q, dq/dx_1 .. dq/dx_3N, Laplacian q).  Linear
// maps act on all rows alike (they run as matrix products in fn_gemm.hip);
// an element-wise f maps value a to f(a), tangent t to f'(a) t and Laplacian
// l to f'(a) l + f''(a) sum_c t_c^2.
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

// ---------------------------------------------------------------------------
// parameter packing into the transposed operand layouts of the products
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void put_w(int mode, void *base, int64_t part, int64_t idx, T v)
{
    if (mode == GEMM_F64) {
        ((double *)base)[idx] = (double)v;
    } else if (mode == GEMM_F32) {
        ((float *)base)[idx] = (float)v;
    } else {
        // BF16 parts, round to nearest even: v = p0 + p1 + ... (each rounds the rest)
        const int np = weight_parts(mode);
        float r = (float)v;
        for (int q = 0; q < np; ++q) {
            uint32_t u = __float_as_uint(r);
            uint32_t h = (u & 0x7fffffffu) > 0x7f800000u ? ((u >> 16) | 0x40u) : ((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
            ((uint16_t *)base)[q * part + idx] = (uint16_t)h;
            r = r - __uint_as_float(h << 16);
        }
    }
}

// Element t of a layer block.  Wx [w1][HWl + GWl]: per-electron inputs
// [h_i | g_i_up | g_i_dn]; Wg [w1][2 HWl]: per-walker inputs [g_up | g_dn].
template <typename T>
__device__ inline void pack_layer_elem(const T *theta, const PackSeg &g, int64_t t)
{
    const int kx = g.HWl + g.GWl, kg = 2 * g.HWl;
    const int64_t nx = (int64_t)g.w1 * kx, ng = (int64_t)g.w1 * kg;
    if (t < nx) {
        const int ti = (int)t, o = ti / kx, k = ti - o * kx;
        int row = -1;
        if (k < g.dh) row = k;
        else if (k >= g.HWl && k < g.HWl + 2 * g.dp) row = 3 * g.dh + (k - g.HWl);
        T v = row >= 0 ? theta[g.off + (int64_t)row * g.w1 + o] : T(0);
        if (g.round) v = (T)bf16_round((float)v);
        put_w<T>(g.mode, g.d0, nx, t, v);
    } else {
        const int64_t u = t - nx;
        const int ui = (int)u, o = ui / kg, k = ui - o * kg;
        int row = -1;
        if (k < g.dh) row = g.dh + k;
        else if (k >= g.HWl && k < g.HWl + g.dh) row = 2 * g.dh + (k - g.HWl);
        T v = row >= 0 ? theta[g.off + (int64_t)row * g.w1 + o] : T(0);
        if (g.round) v = (T)bf16_round((float)v);
        put_w<T>(g.mode2, g.d1, ng, u, v);
    }
}

// Element t of a head block: Wh [K n][W1p] from w [w1][K n]
template <typename T>
__device__ inline void pack_head_elem(const T *theta, const PackSeg &g, int64_t t)
{
    const int64_t n = (int64_t)g.kn * g.W1p;
    const int ti = (int)t, col = ti / g.W1p, k = ti - col * g.W1p;
    T v = k < g.w1 ? theta[g.off + (int64_t)k * g.kn + col] : T(0);
    if (g.round) v = (T)bf16_round((float)v);
    put_w<T>(g.mode, g.d0, n, t, v);
}

// Element t of a pair block (FP32, matrix-core pair kernel layout)
template <typename T>
__device__ inline void pack_pair_elem(const T *theta, const PackSeg &g, int64_t t)
{
    T v = T(0);
    if (t < (int64_t)g.wc * g.ks) {
        const int ti = (int)t, o = ti / g.ks, k = ti - o * g.ks;
        if (o < g.w2 && k < g.dp) v = theta[g.off + (int64_t)k * g.w2 + o];
    } else {
        const int o = (int)(t - (int64_t)g.wc * g.ks);
        if (o < g.w2) v = theta[g.off2 + o];
    }
    ((float *)g.d0)[t] = (float)v;
}

// every forward operand block in one launch; segment q takes the
// workgroups [bbegin_q, bbegin_(q+1)), one element of its count_q per thread
// (the segment is the same for the whole workgroup)
template <typename T>
__global__ __launch_bounds__(256) void k_pack(const T *theta, PackList pl)
{
    int q = 0;
    while (q + 1 < pl.n && (int)blockIdx.x >= pl.seg[q + 1].bbegin) ++q;
    const PackSeg &g = pl.seg[q];
    const int64_t t = (int64_t)((int)blockIdx.x - g.bbegin) * blockDim.x + threadIdx.x;
    if (t >= g.count) return;
    if (g.kind == 0) pack_layer_elem<T>(theta, g, t);
    else if (g.kind == 1) pack_head_elem<T>(theta, g, t);
    else if (g.kind == 2) pack_pair_elem<T>(theta, g, t);
    else ((T *)g.d0)[t] = (T)bf16_round((float)theta[g.off + t]);
}

// ---------------------------------------------------------------------------
// electron-nucleus input features [r_i - R_m, |r_i - R_m|] with their rows
// ---------------------------------------------------------------------------
// four consecutive columns of a row (16-byte aligned)
__device__ inline void store4(float *p, float a, float b, float c, float d) { *(float4 *)p = make_float4(a, b, c, d); }
__device__ inline void store4(double *p, double a, double b, double c, double d)
{
    ((double2 *)p)[0] = make_double2(a, b);
    ((double2 *)p)[1] = make_double2(c, d);
}

// One item per (walker, electron, row t, nucleus m): the four columns
// [r_i - R_m, |r_i - R_m|] of that row, the distance formed once in FP64.
// Columns of m >= M (padding up to HW0) are zero.
template <typename T>
__global__ __launch_bounds__(256) void k_features(Sys s, const double *x, int64_t B, int TR, int HW0, int64_t ldh,
                                                  T *H, T *G)
{
    const int mq = HW0 / 4;
    const int n3 = 3 * s.N;
    const int64_t total = B * s.N * TR * mq;
    // then the spin means of these rows for the first layer: G[w TR + t] =
    // [g_up | g_dn] (row width 2 HW0) for t up to the Laplacian row, each
    // the FP rounding of the features summed over the spin's electrons in
    // order and scaled by 1 / n, as the spin-mean kernel forms them
    const int live = TR == 1 ? 1 : n3 + 2;
    const int64_t gtotal = G ? B * live * 2 * mq : 0;
    for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < total + gtotal;
         it += (int64_t)gridDim.x * blockDim.x) {
        if (it >= total) {
            const int64_t ig = it - total;
            const int q = (int)(ig % (2 * mq));
            const int64_t wt = ig / (2 * mq);             // walker * live + t
            const int64_t w = wt / live;
            const int t = (int)(wt - w * live);
            const int sp = q >= mq, m = q - sp * mq;
            const int n = sp ? s.N - s.nu : s.nu, j0 = sp ? s.nu : 0;
            const T inv = n > 0 ? T(1) / T(n) : T(0);
            T v[4] = {T(0), T(0), T(0), T(0)};
            if (m < s.M && n > 0) {
                int e = -1, a = -1;                       // tangent row of electron e's coordinate a
                if (t >= 1 && t <= n3) { e = (t - 1) / 3; a = t - 1 - 3 * e; }
                for (int j = j0; j < j0 + n; ++j) {
                    if (e >= 0 && j != e) continue;       // other electrons' tangent rows are zero
                    const double *xj = x + (w * s.N + j) * 3;
                    const double d0 = xj[0] - s.R[m][0], d1 = xj[1] - s.R[m][1], d2 = xj[2] - s.R[m][2];
                    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    if (t == 0) {
                        v[0] += (T)d0; v[1] += (T)d1; v[2] += (T)d2; v[3] += (T)r;
                    } else if (t == n3 + 1) {
                        v[3] += (T)(2.0 / r);
                    } else {
                        const double da = a == 0 ? d0 : (a == 1 ? d1 : d2);
                        v[a] += T(1);
                        v[3] += (T)(da / r);
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) v[c] *= inv;
            }
            store4(G + (w * TR + t) * (2 * (int64_t)HW0) + sp * HW0 + 4 * m, v[0], v[1], v[2], v[3]);
            continue;
        }
        const int m = (int)(it % mq);
        const int64_t row = it / mq;                  // (walker * N + electron) * TR + t
        const int t = (int)(row % TR);
        const int64_t wi = row / TR;
        const int i = (int)(wi % s.N);
        T v[4] = {T(0), T(0), T(0), T(0)};
        if (m < s.M && t <= n3 + 1) {
            int a = -1;                               // tangent row of this electron's coordinate a
            if (t >= 1 && t <= n3) {
                const int c = t - 1, e = c / 3;
                if (e == i) a = c - 3 * e;
            }
            if (t == 0 || t == n3 + 1 || a >= 0) {
                const double *xi = x + wi * 3;
                const double d0 = xi[0] - s.R[m][0], d1 = xi[1] - s.R[m][1], d2 = xi[2] - s.R[m][2];
                const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                if (t == 0) {
                    v[0] = (T)d0; v[1] = (T)d1; v[2] = (T)d2; v[3] = (T)r;
                } else if (t == n3 + 1) {
                    v[3] = (T)(2.0 / r);
                } else {
                    const double da = a == 0 ? d0 : (a == 1 ? d1 : d2);
                    v[a] = T(1);
                    v[3] = (T)(da / r);
                }
            }
        }
        store4(H + row * ldh + 4 * m, v[0], v[1], v[2], v[3]);
    }
}

// ---------------------------------------------------------------------------
// two-electron stream: a workgroup takes WB consecutive (walker, electron i)
// and runs their pairs (i, j) through all pair layers, writing the spin means
// g_i_up, g_i_dn of every layer as dense rows.  A pair feature depends on r_i
// and r_j only, so a pair carries R = 8 rows: value, d/dr_i (3), d/dr_j (3),
// Laplacian.  The pair weights are staged in LDS once per workgroup, padded
// to multiples of 4 (zero rows and columns); a thread owns one pair and 4
// output columns for all R rows.
// ---------------------------------------------------------------------------
template <typename T, bool FL>
__device__ void write_pair_means(const Sys &s, const T *S, int wp, int ps, int dp, int i, int TR, int GWl, int64_t ldg,
                                 T *gi)
{
    constexpr int R = FL ? 8 : 1;
    const int n3 = 3 * s.N;
    const int rows = FL ? TR : 1;
    if constexpr (std::is_same<T, float>::value) {
        if (dp % 4 == 0) {
            // a thread keeps four columns of one spin block (float4 reads of
            // the 16-byte aligned pair rows, float4 stores) and walks rows
            const int cqn = GWl / 4, tstep = blockDim.x / cqn;
            if ((int)threadIdx.x >= tstep * cqn) return;
            const int col = 4 * ((int)threadIdx.x % cqn);
            const bool live = col < 2 * dp;
            const int sp = live ? col / dp : 0, o = live ? col - sp * dp : 0;
            const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
            const float inv = n > 0 ? 1.f / (float)n : 0.f;
            auto ld4 = [&](int j, int r) { return *(const float4 *)(S + j * ps + r * wp + o); };
            for (int t = threadIdx.x / cqn; t < rows; t += tstep) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (live && n > 0 && t <= n3 + 1) {
                    int r = -1;                   // summed row of every pair of the spin, or -1
                    int e = -1;                   // single pair (i, e) for another electron's direction
                    if (t == 0 || t == n3 + 1) {
                        r = t == 0 ? 0 : R - 1;
                    } else {
                        const int c = t - 1, ee = c / 3, a = c - 3 * ee;
                        if (ee == i) r = 1 + a;
                        else if (ee >= j0 && ee < j0 + n) { e = ee; r = 4 + a; }
                    }
                    if (e >= 0) {
                        const float4 q = ld4(e, r);
                        v = make_float4(q.x * inv, q.y * inv, q.z * inv, q.w * inv);
                    } else if (r >= 0) {
                        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                        for (int j = j0; j < j0 + n; ++j) {
                            const float4 q = ld4(j, r);
                            acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w += q.w;
                        }
                        v = make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w * inv);
                    }
                }
                *(float4 *)(gi + (int64_t)t * ldg + col) = v;
            }
            return;
        }
    }
    // a thread keeps one column and walks rows; the first (blockDim / GWl) GWl threads take part
    const int tstep = blockDim.x / GWl;
    if ((int)threadIdx.x >= tstep * GWl) return;
    const int col = threadIdx.x % GWl;
    const bool live = col < 2 * dp;
    const int sp = live ? col / dp : 0, o = live ? col - sp * dp : 0;
    const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
    const T inv = n > 0 ? T(1) / T(n) : T(0);
    for (int t = threadIdx.x / GWl; t < rows; t += tstep) {
        T v = T(0);
        if (live && n > 0 && t <= n3 + 1) {
            if (t == 0 || t == n3 + 1) {
                const int r = t == 0 ? 0 : R - 1;
                T acc = T(0);
                for (int j = j0; j < j0 + n; ++j) acc += S[j * ps + r * wp + o];
                v = acc * inv;
            } else {
                const int c = t - 1, e = c / 3, a = c - 3 * e;
                if (e == i) {
                    T acc = T(0);
                    for (int j = j0; j < j0 + n; ++j) acc += S[j * ps + (1 + a) * wp + o];
                    v = acc * inv;
                } else if (e >= j0 && e < j0 + n) {
                    v = S[e * ps + (4 + a) * wp + o] * inv;
                }
            }
        }
        gi[(int64_t)t * ldg + col] = v;
    }
}

// The same rows for the nwi (walker, electron) rows of a workgroup at once,
// FP32 with dp a multiple of 4: one item per (row, output row t, four
// columns), so every thread takes part however few rows each has.  S holds
// row bb at S + bb * per; gi0 is the layer's output base.
template <bool FL>
__device__ void write_pair_means_wg(const Sys &s, const float *S, int per, int wp, int ps, int dp, int64_t wi0,
                                    int nwi, int TR, int GWl, int64_t ldg, float *gi0)
{
    constexpr int R = FL ? 8 : 1;
    // rows value .. Laplacian only: the padding rows of TR are never read
    // (every product over these rows reads its live rows only)
    const int n3 = 3 * s.N, rows = FL ? TR : 1, live_rows = FL ? n3 + 2 : 1, cqn = GWl / 4;
    const int items = nwi * live_rows * cqn;
    // item it = (bb live_rows + t) cqn + col / 4.  When cqn divides the
    // workgroup size a thread keeps its column and its (row, t) advances by
    // a fixed step, so the index arithmetic is done once
    const bool fixed_col = (int)blockDim.x % cqn == 0;
    const int rstep = (int)blockDim.x / cqn;
    const int i0 = (int)(wi0 % s.N);
    int t = 0, bb = 0, ccol = 0;
    if (fixed_col) {
        const int rt0 = (int)threadIdx.x / cqn;
        ccol = 4 * ((int)threadIdx.x - rt0 * cqn);
        t = rt0 % live_rows;
        bb = rt0 / live_rows;
    }
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        int col;
        if (fixed_col) {
            col = ccol;
        } else {
            const int rt = it / cqn;
            col = 4 * (it - rt * cqn);
            t = rt % live_rows;
            bb = rt / live_rows;
        }
        const int64_t wi = wi0 + bb;
        int i = i0 + bb;                               // (wi0 + bb) mod N, bb < nwi
        while (i >= s.N) i -= s.N;
        const float *Sb = S + (int64_t)bb * per;
        const bool live = col < 2 * dp;
        const int sp = live ? col / dp : 0, o = live ? col - sp * dp : 0;
        const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
        const float inv = n > 0 ? 1.f / (float)n : 0.f;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live && n > 0 && t <= n3 + 1) {
            int r = -1, e = -1;
            if (t == 0 || t == n3 + 1) {
                r = t == 0 ? 0 : R - 1;
            } else {
                const int c = t - 1, ee = c / 3, a = c - 3 * ee;
                if (ee == i) r = 1 + a;
                else if (ee >= j0 && ee < j0 + n) { e = ee; r = 4 + a; }
            }
            if (e >= 0) {
                const float4 q = *(const float4 *)(Sb + e * ps + r * wp + o);
                v = make_float4(q.x * inv, q.y * inv, q.z * inv, q.w * inv);
            } else if (r >= 0) {
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                for (int j = j0; j < j0 + n; ++j) {
                    const float4 q = *(const float4 *)(Sb + j * ps + r * wp + o);
                    acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w += q.w;
                }
                v = make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w * inv);
            }
        }
        *(float4 *)(gi0 + (wi * rows + t) * ldg + col) = v;
        if (fixed_col) {
            t += rstep;
            while (t >= live_rows) {
                t -= live_rows;
                ++bb;
            }
        }
    }
}

// OC consecutive LDS elements (16-, 8- or 4-byte aligned for FP32)
template <typename T, int OC>
__device__ inline void lds_ld(const T *p, T (&v)[OC])
{
#pragma unroll
    for (int c = 0; c < OC; ++c) v[c] = p[c];
}

template <>
__device__ inline void lds_ld<float, 4>(const float *p, float (&v)[4])
{
    const float4 q = *(const float4 *)p;
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}

template <>
__device__ inline void lds_ld<float, 2>(const float *p, float (&v)[2])
{
    const float2 q = *(const float2 *)p;
    v[0] = q.x; v[1] = q.y;
}

template <typename T, int OC>
__device__ inline void lds_st(T *p, const T (&v)[OC])
{
#pragma unroll
    for (int c = 0; c < OC; ++c) p[c] = v[c];
}

template <>
__device__ inline void lds_st<float, 4>(float *p, const float (&v)[4])
{
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
}

template <>
__device__ inline void lds_st<float, 2>(float *p, const float (&v)[2])
{
    *(float2 *)p = make_float2(v[0], v[1]);
}

// explicit fused multiply-add, so that every launch shape of the pair kernel
// rounds alike
template <typename T>
__device__ inline T fmat(T a, T b, T c);
template <>
__device__ inline float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ inline double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// padded pair-weight block of layer l in LDS: [dp4][w2p] then bias [w2p]
__host__ __device__ inline int pair_w_offset(const Sys &s, int l)
{
    const int w2p = round_up(s.w2, 4);
    int o = 0;
    for (int q = 0; q < l; ++q) o += (round_up(layer_dp(s, q), 4) + 1) * w2p;
    return o;
}

template <typename T, bool FL, int OC>
__global__ __launch_bounds__(256) void k_pair_stream(Sys s, const double *x, const T *theta, ParamLayout P, int64_t B,
                                                     int TR, int64_t ldg, int64_t gi_layer_stride, int GW0, int GW1,
                                                     int WB, T *GI)
{
    constexpr int R = FL ? 8 : 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int w2p = round_up(s.w2, 4);
    const int wp = w2p > 4 ? w2p : 4;                     // LDS row width of a pair
    const int ps = R * wp + 128 / (int)sizeof(T);         // one pair; a 128-byte skew puts neighbouring pairs on other banks
    const int per = s.N * ps;                             // one (walker, electron) in LDS
    T *S0 = (T *)smem_raw;
    T *S1 = S0 + (int64_t)WB * per;
    T *Wsm = S1 + (int64_t)WB * per;
    const int tid = threadIdx.x;
    for (int l = 0; l + 1 < s.L; ++l) {
        const int dp = layer_dp(s, l), dp4 = round_up(dp, 4);
        T *Wl = Wsm + pair_w_offset(s, l);
        for (int q = tid; q < (dp4 + 1) * w2p; q += blockDim.x) {
            const int k = q / w2p, o = q % w2p;
            T v = T(0);
            if (o < s.w2) {
                if (k < dp) v = theta[P.W2[l] + (int64_t)k * s.w2 + o];
                else if (k == dp4) v = theta[P.c2[l] + o];
            }
            Wl[q] = v;
        }
    }
    const int64_t wi0 = (int64_t)blockIdx.x * WB;
    const int nwi = B * s.N - wi0 < WB ? (int)(B * s.N - wi0) : WB;
    const int rows = FL ? TR : 1;

    // layer-0 pair features (zero rows first, then the nonzero entries)
    for (int q = tid; q < nwi * per; q += blockDim.x) S0[q] = T(0);
    __syncthreads();
    for (int q = tid; q < nwi * s.N; q += blockDim.x) {
        const int bb = q / s.N, j = q % s.N;
        const int64_t wi = wi0 + bb, w = wi / s.N;
        const int i = (int)(wi % s.N);
        const double *xw = x + w * 3 * s.N;
        T *p = S0 + (int64_t)bb * per + j * ps;
        if (j == i) continue;
        double d[3] = {xw[3 * i] - xw[3 * j], xw[3 * i + 1] - xw[3 * j + 1], xw[3 * i + 2] - xw[3 * j + 2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int c = 0; c < 3; ++c) p[c] = (T)d[c];
        p[3] = (T)r;
        if constexpr (FL) {
            for (int c = 0; c < 3; ++c) {
                p[(1 + c) * wp + c] = T(1);
                p[(1 + c) * wp + 3] = (T)(d[c] / r);
                p[(4 + c) * wp + c] = T(-1);
                p[(4 + c) * wp + 3] = (T)(-d[c] / r);
            }
            p[7 * wp + 3] = (T)(4.0 / r);
        }
    }
    __syncthreads();
    for (int bb = 0; bb < nwi; ++bb) {
        const int64_t wi = wi0 + bb;
        write_pair_means<T, FL>(s, S0 + (int64_t)bb * per, wp, ps, 4, (int)(wi % s.N), TR, GW0, ldg, GI + wi * rows * ldg);
    }
    const int ocn = w2p / OC;                             // column groups of a pair
    for (int l = 0; l + 1 < s.L; ++l) {
        __syncthreads();
        const int dp4 = round_up(layer_dp(s, l), 4);
        const T *Wl = Wsm + pair_w_offset(s, l);
        const T *cl = Wl + dp4 * w2p;
        for (int q = tid; q < nwi * s.N * ocn; q += blockDim.x) {
            const int bb = q / (s.N * ocn), rem = q % (s.N * ocn);
            const int j = rem / ocn, o0 = OC * (rem % ocn);
            const T *in = S0 + (int64_t)bb * per + j * ps;
            T acc[R][OC];
            T bias[OC];
            lds_ld<T, OC>(cl + o0, bias);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < OC; ++c) acc[r][c] = r == 0 ? bias[c] : T(0);
            for (int k = 0; k < dp4; k += 4) {
                T wv[4][OC];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) lds_ld<T, OC>(Wl + (k + kk) * w2p + o0, wv[kk]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T xv[4];
                    lds_ld<T, 4>(in + r * wp + k, xv);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int c = 0; c < OC; ++c) acc[r][c] = fmat(xv[kk], wv[kk][c], acc[r][c]);
                }
            }
            T *out = S1 + (int64_t)bb * per + j * ps;
            T y0[OC], dd[OC], src[OC];
#pragma unroll
            for (int c = 0; c < OC; ++c) {
                y0[c] = tanh(acc[0][c]);
                dd[c] = fmat(-y0[c], y0[c], T(1));
                src[c] = T(0);
            }
            // rows stored OC columns at a time; residual rows read likewise
#pragma unroll
            for (int r = 0; r < R; ++r) {
                T res[OC];
#pragma unroll
                for (int c = 0; c < OC; ++c) res[c] = T(0);
                if (l >= 1) lds_ld<T, OC>(in + r * wp + o0, res);
                T v[OC];
#pragma unroll
                for (int c = 0; c < OC; ++c) {
                    if (r == 0) {
                        v[c] = y0[c] + res[c];
                    } else if (r < 7) {
                        src[c] = fmat(acc[r][c], acc[r][c], src[c]);
                        v[c] = fmat(dd[c], acc[r][c], res[c]);
                    } else {
                        const T q = T(-2) * y0[c] * dd[c];
                        v[c] = fmat(dd[c], acc[R - 1][c], fmat(q, src[c], res[c]));
                    }
                }
                lds_st<T, OC>(out + r * wp + o0, v);
            }
        }
        __syncthreads();
        T *t = S0; S0 = S1; S1 = t;
        for (int bb = 0; bb < nwi; ++bb) {
            const int64_t wi = wi0 + bb;
            write_pair_means<T, FL>(s, S0 + (int64_t)bb * per, wp, ps, s.w2, (int)(wi % s.N), TR, GW1, ldg,
                                    GI + (int64_t)(l + 1) * gi_layer_stride + wi * rows * ldg);
        }
    }
}

// ---------------------------------------------------------------------------
// two-electron stream on the matrix cores, FP32 operands: the layers of
// k_pair_stream with each pair layer a product of 16-row blocks of pair rows
// (two pairs of 8 forward-Laplacian rows, or 16 value rows) with the
// transposed weights, v_mfma_f32_16x16x4f32 with four reduction steps per
// float4 read.  A wave owns whole row blocks and updates them in place after
// all of its reads.  Forward-Laplacian epilogue: lane groups 0/2 hold rows
// 0-3 of a pair (value, tangents 1-3), groups 1/3 rows 4-7 (tangents 4-6,
// Laplacian); one exchange between the two (lane ^ 16) gives both the tanh
// value and the source sum_c dz_c^2.
// LDS: rows of wc + 4 floats (wc = w2 rounded up to 16), pair j of
// (walker, electron) b at rows (b N + j) R ..; per pair layer the transposed
// weights Wt[wc][KP + 4] (KP = d_p rounded up to 16), then the bias [wc].
// ---------------------------------------------------------------------------
template <bool FL>
__global__ __launch_bounds__(256) void k_pair_mfma(Sys s, const double *x, const float *__restrict__ Wpk,
                                                   int64_t B, int TR, int64_t ldg, int64_t gi_layer_stride, int GW0,
                                                   int GW1, int WB, float *GI)
{
    constexpr int R = FL ? 8 : 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int wc = round_up(s.w2, 16), RS = wc + 4, ps = R * RS, per = s.N * ps;
    const int ncb = wc / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, li = lane & 15;
    const int64_t wi0 = (int64_t)blockIdx.x * WB;
    const int nwi = B * s.N - wi0 < WB ? (int)(B * s.N - wi0) : WB;
    const int nrow = nwi * s.N * R;                       // pair rows held here
    const int nblk = (nrow + 15) / 16;
    const int rows_alloc = round_up(WB * s.N * R, 16);
    float *S = (float *)smem_raw;
    float *Wsm = S + (int64_t)rows_alloc * RS;

    // packed weights: a plain copy (the block is a multiple of 16 floats)
    const int wtot = pair_mfma_woff(s, s.L > 1 ? s.L - 1 : 0);
    for (int q = 4 * tid; q < wtot; q += 4 * blockDim.x) *(float4 *)(Wsm + q) = *(const float4 *)(Wpk + q);
    for (int q = 4 * tid; q < rows_alloc * RS; q += 4 * blockDim.x) *(float4 *)(S + q) = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // layer-0 pair features
    for (int q = tid; q < nwi * s.N; q += blockDim.x) {
        const int bb = q / s.N, j = q % s.N;
        const int64_t wi = wi0 + bb, w = wi / s.N;
        const int i = (int)(wi % s.N);
        if (j == i) continue;
        const double *xw = x + w * 3 * s.N;
        float *p = S + (int64_t)bb * per + j * ps;
        const double d[3] = {xw[3 * i] - xw[3 * j], xw[3 * i + 1] - xw[3 * j + 1], xw[3 * i + 2] - xw[3 * j + 2]};
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int c = 0; c < 3; ++c) p[c] = (float)d[c];
        p[3] = (float)r;
        if constexpr (FL) {
            for (int c = 0; c < 3; ++c) {
                p[(1 + c) * RS + c] = 1.f;
                p[(1 + c) * RS + 3] = (float)(d[c] / r);
                p[(4 + c) * RS + c] = -1.f;
                p[(4 + c) * RS + 3] = (float)(-d[c] / r);
            }
            p[7 * RS + 3] = (float)(4.0 / r);
        }
    }
    __syncthreads();
    write_pair_means_wg<FL>(s, S, per, RS, ps, 4, wi0, nwi, TR, GW0, ldg, GI);
    for (int l = 0; l + 1 < s.L; ++l) {
        __syncthreads();
        const int KP = pair_mfma_kp(s, l), KS = KP + 4;
        const float *Wl = Wsm + pair_mfma_woff(s, l);
        const float *bl = Wl + wc * KS;
        const bool resid = l >= 1;
        for (int blk = wave; blk < nblk; blk += 4) {
            const int r0 = blk * 16;
            f32x4 acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const float bv = cb < ncb ? bl[cb * 16 + li] : 0.f;
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[cb][e] = (!FL || ((g & 1) == 0 && e == 0)) ? bv : 0.f;
            }
            const float *arow = S + (int64_t)(r0 + li) * RS + 4 * g;
            for (int kb = 0; kb < KP; kb += 16) {
                const float4 a4 = *(const float4 *)(arow + kb);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    if (cb < ncb) {
                        const float4 b4 = *(const float4 *)(Wl + (cb * 16 + li) * KS + kb + 4 * g);
                        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b4.x, acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b4.y, acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b4.z, acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b4.w, acc[cb], 0, 0, 0);
                    }
                }
            }
            // every read of this block is done: write its rows in place
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (cb >= ncb) continue;
                const int col = cb * 16 + li;
                float *o = S + (int64_t)(r0 + 4 * g) * RS + col;
                float res[4], v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) res[e] = resid ? o[e * RS] : 0.f;
                const float a0 = acc[cb][0], a1 = acc[cb][1], a2 = acc[cb][2], a3 = acc[cb][3];
                if constexpr (FL) {
                    const bool ev = (g & 1) == 0;
                    const float part = ev ? fmat(a3, a3, fmat(a2, a2, a1 * a1)) : fmat(a2, a2, fmat(a1, a1, a0 * a0));
                    const float y0c = tanhf(a0);
                    const float part_o = __shfl_xor(part, 16);
                    const float y0_o = __shfl_xor(y0c, 16);
                    const float y0 = ev ? y0c : y0_o;
                    const float src = ev ? part + part_o : part_o + part;
                    const float dd = fmat(-y0, y0, 1.f);
                    if (ev) {
                        v[0] = y0 + res[0];
                        v[1] = fmat(dd, a1, res[1]);
                        v[2] = fmat(dd, a2, res[2]);
                        v[3] = fmat(dd, a3, res[3]);
                    } else {
                        v[0] = fmat(dd, a0, res[0]);
                        v[1] = fmat(dd, a1, res[1]);
                        v[2] = fmat(dd, a2, res[2]);
                        v[3] = fmat(dd, a3, fmat(-2.f * y0 * dd, src, res[3]));
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = tanhf(acc[cb][e]) + res[e];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r0 + 4 * g + e < nrow) o[e * RS] = v[e];
            }
        }
        __syncthreads();
        write_pair_means_wg<FL>(s, S, per, RS, ps, s.w2, wi0, nwi, TR, GW1, ldg,
                                GI + (int64_t)(l + 1) * gi_layer_stride);
    }
}

// ---------------------------------------------------------------------------
// spin means of the one-electron stream: G[w][t] = [g_up | g_dn] for the rows
// t of each walker up to its Laplacian row (live); one item
// per (walker row, output column), FP32 rows four columns per item
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_spin_mean(const T *__restrict__ H, int64_t ldh, int64_t B, int N, int nu,
                                                   int TR, int live, int dh, int HWl, T *__restrict__ G)
{
    const int nd = N - nu;
    const T iu = nu > 0 ? T(1) / T(nu) : T(0), id = nd > 0 ? T(1) / T(nd) : T(0);
    const int64_t total = B * live * 2 * HWl;
    for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(it % (2 * HWl));
        const int64_t wl = it / (2 * HWl);            // walker * live + t
        const int64_t w = wl / live;
        const int t = (int)(wl - w * live);
        const int64_t wt = w * TR + t;
        const T *h0 = H + (w * N * TR + t) * ldh;
        const int64_t jstride = (int64_t)TR * ldh;
        const int sp = col >= HWl, k = col - sp * HWl;
        T v = T(0);
        if (k < dh) {
            const int j0 = sp ? nu : 0, j1 = sp ? N : nu;
            // four rows requested at once, added in electron order
            int j = j0;
            for (; j + 4 <= j1; j += 4) {
                const T a0 = h0[j * jstride + k], a1 = h0[(j + 1) * jstride + k];
                const T a2 = h0[(j + 2) * jstride + k], a3 = h0[(j + 3) * jstride + k];
                v += a0; v += a1; v += a2; v += a3;
            }
            for (; j < j1; ++j) v += h0[j * jstride + k];
            v *= sp ? id : iu;
        }
        G[wt * 2 * HWl + col] = v;
    }
}

template <>
__global__ __launch_bounds__(256) void k_spin_mean<float>(const float *__restrict__ H, int64_t ldh, int64_t B, int N,
                                                          int nu, int TR, int live, int dh, int HWl,
                                                          float *__restrict__ G)
{
    const int nd = N - nu;
    const float iu = nu > 0 ? 1.f / nu : 0.f, id = nd > 0 ? 1.f / nd : 0.f;
    const int cq = HWl / 2;                           // float4s in [g_up | g_dn] (HWl is a multiple of 32)
    const int64_t total = B * live * cq;
    for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int col = 4 * (int)(it % cq);
        const int64_t wl = it / cq;                   // walker * live + t
        const int64_t w = wl / live;
        const int t = (int)(wl - w * live);
        const int64_t wt = w * TR + t;
        const float *h0 = H + (w * N * TR + t) * ldh;
        const int64_t jstride = (int64_t)TR * ldh;
        const int sp = col >= HWl, k = col - sp * HWl;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < dh) {
            const int j0 = sp ? nu : 0, j1 = sp ? N : nu;
            // up to four rows requested at once, added in electron order
            for (int jb = j0; jb < j1; jb += 4) {
                float4 h[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    h[u] = jb + u < j1 ? *(const float4 *)(h0 + (jb + u) * jstride + k) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (jb + u < j1) { v.x += h[u].x; v.y += h[u].y; v.z += h[u].z; v.w += h[u].w; }
            }
            const float sc = sp ? id : iu;
            v.x *= sc; v.y *= sc; v.z *= sc; v.w *= sc;
            // columns dh.. of the padded block are zero in H, so whole float4s are safe
        }
        *(float4 *)(G + wt * 2 * HWl + col) = v;
    }
}

// ---------------------------------------------------------------------------
// layer epilogue: z = X + P (per-walker part) + b (value row), y = tanh(z) in
// forward-Laplacian form, plus the residual h_i when widths match (l >= 1).
// ---------------------------------------------------------------------------
template <typename T, bool FL>
__global__ __launch_bounds__(256) void k_layer_epi(const T *__restrict__ X, const T *__restrict__ Pw,
                                                   const T *__restrict__ bias, const T *__restrict__ Hin,
                                                   T *__restrict__ Hout, int64_t ldh, int N, int TR, int n3, int w1,
                                                   int W1p, int resid, T *__restrict__ Tout)
{
    const int wi = blockIdx.x;              // walker * N + electron
    const int w = wi / N;
    const int64_t r0 = (int64_t)wi * TR;
    for (int o = threadIdx.x; o < W1p; o += blockDim.x) {
        if (o >= w1) {
            for (int t = 0; t < TR; ++t) Hout[(r0 + t) * ldh + o] = T(0);
            continue;
        }
        const T *xp = X + r0 * w1 + o;
        const T *pp = Pw + (int64_t)w * TR * w1 + o;
        const T z0 = xp[0] + pp[0] + bias[o];
        const T y0 = tanh(z0);
        const T d = T(1) - y0 * y0;
        Hout[r0 * ldh + o] = y0 + (resid ? Hin[r0 * ldh + o] : T(0));
        if (Tout) Tout[r0 * w1 + o] = y0;
        if (FL) {
            T src = T(0);
            for (int t = 1; t <= n3; ++t) {
                const T z = xp[(int64_t)t * w1] + pp[(int64_t)t * w1];
                src += z * z;
                Hout[(r0 + t) * ldh + o] = d * z + (resid ? Hin[(r0 + t) * ldh + o] : T(0));
            }
            const int tl = n3 + 1;
            const T zl = xp[(int64_t)tl * w1] + pp[(int64_t)tl * w1];
            Hout[(r0 + tl) * ldh + o] = d * zl - T(2) * y0 * d * src + (resid ? Hin[(r0 + tl) * ldh + o] : T(0));
            for (int t = tl + 1; t < TR; ++t) Hout[(r0 + t) * ldh + o] = T(0);
        }
    }
}

// ---------------------------------------------------------------------------
// orbitals x envelope (Eq. 4): phi_i(j) = (w_i . h_j + g_i) sum_m pi_im
// exp(-|Sigma_im (r_j - R_m)|).  The envelope depends on r_j only, so its
// derivatives are local to the three coordinates of electron j:
//   q = |Sigma d|, grad q = S d / q with S = Sigma^T Sigma,
//   lap q = (tr S - |S d|^2 / q^2) / q, grad e = -e grad q,
//   lap e = e (|grad q|^2 - lap q); lap(a e) = e lap a + a lap e + 2 grad a . grad e.
// Output Phi[w][k][t][i][jj] (rows t = value, 3N tangents, Laplacian).
// ---------------------------------------------------------------------------
// One nucleus' term of orbital column col's envelope at electron position
// xj: em = pi exp(-q) added to env, and with FL its contributions to the
// electron's gradient and Laplacian of the envelope (all FP64).
//   anisotropic: q = |Sigma d|, grad q = S d / q, S = Sigma^T Sigma,
//                lap q = (tr S - |S d|^2 / q^2) / q;
//   isotropic (Sigma = sigma I): q = |sigma| r with r = |d|,
//                grad q = |sigma| d / r, |grad q|^2 = sigma^2, lap q = 2 |sigma| / r.
template <typename T, bool FL>
__device__ __forceinline__ void env_add(const Sys &s, const T *theta, int64_t piof, int64_t sigof, int col, int m,
                                        const double *xj, double &env, double (&ge)[3], double &le)
{
    const double d[3] = {xj[0] - s.R[m][0], xj[1] - s.R[m][1], xj[2] - s.R[m][2]};
    if (s.iso) {
        const double sg = fabs((double)theta[sigof + (int64_t)col * s.M + m]);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double em = (double)theta[piof + (int64_t)col * s.M + m] * exp(-(sg * r));
        env += em;
        if constexpr (FL) {
            const double gr = sg / r;
            for (int a = 0; a < 3; ++a) ge[a] -= em * gr * d[a];
            le += em * (sg * sg - 2.0 * gr);
        }
        return;
    }
    const T *Sgp = theta + sigof + ((int64_t)col * s.M + m) * 9;
    double sd[3], ad[3], Sg[9];
    for (int e = 0; e < 9; ++e) Sg[e] = (double)Sgp[e];
    for (int p = 0; p < 3; ++p) sd[p] = Sg[3 * p] * d[0] + Sg[3 * p + 1] * d[1] + Sg[3 * p + 2] * d[2];
    for (int a = 0; a < 3; ++a) ad[a] = Sg[a] * sd[0] + Sg[3 + a] * sd[1] + Sg[6 + a] * sd[2];
    const double qd = sqrt(sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2]);
    const double em = (double)theta[piof + (int64_t)col * s.M + m] * exp(-qd);
    env += em;
    if constexpr (FL) {
        double trS = 0.0;
        for (int e = 0; e < 9; ++e) trS += Sg[e] * Sg[e];
        const double iq = 1.0 / qd;
        const double ad2 = ad[0] * ad[0] + ad[1] * ad[1] + ad[2] * ad[2];
        const double lq = (trS - ad2 * iq * iq) * iq;
        const double gq2 = ad2 * iq * iq;
        for (int a = 0; a < 3; ++a) ge[a] -= em * ad[a] * iq;
        le += em * (gq2 - lq);
    }
}

template <typename T, bool FL>
__global__ void k_envelope(Sys s, const double *x, const T *theta, int64_t gof, int64_t piof, int64_t sigof, int sp,
                           const T *O, int64_t ldo, int64_t B, int TR, double *Phi)
{
    typedef double E;   // envelope and product rule in FP64 for every precision
    const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
    const int kn = s.K * n;
    const int n3 = 3 * s.N;
    const int64_t total = B * n * kn;
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total; id += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(id % kn);
        const int64_t wj = id / kn;
        const int jj = (int)(wj % n);
        const int64_t w = wj / n;
        const int j = j0 + jj;
        const int k = col / n, io = col % n;
        const double *xj = x + (w * s.N + j) * 3;
        E env = 0.0, ge[3] = {0.0, 0.0, 0.0}, le = 0.0;
        for (int m = 0; m < s.M; ++m) env_add<T, FL>(s, theta, piof, sigof, col, m, xj, env, ge, le);
        const int64_t orow = (w * n + jj) * TR;
        const E a0 = (E)O[orow * ldo + col] + (E)theta[gof + col];
        const int64_t base = ((w * s.K + k) * TR) * n * n + io * n + jj;
        const int64_t tstride = (int64_t)n * n;
        Phi[base] = a0 * env;
        if (FL) {
            for (int c = 0; c < n3; ++c) {
                E v = env * (E)O[(orow + 1 + c) * ldo + col];
                if (c / 3 == j) v += a0 * ge[c % 3];
                Phi[base + (1 + c) * tstride] = v;
            }
            E lap = env * (E)O[(orow + n3 + 1) * ldo + col] + a0 * le;
            for (int a = 0; a < 3; ++a) lap += 2.0 * (E)O[(orow + 1 + 3 * j + a) * ldo + col] * ge[a];
            Phi[base + (n3 + 1) * tstride] = lap;
        }
    }
}

// ---------------------------------------------------------------------------
// determinants: one wave64 per (walker, determinant k) of one spin.  LU with
// partial pivoting in LDS gives sign and log|det A|; then for every
// direction c the columns of M_c = A^-1 dA/dx_c come from LU solves, and
//   d log|det| / dx_c = tr M_c,
//   lap log|det| = tr(A^-1 lap A) - sum_c tr(M_c M_c).
// Record layout per (walker, spin, k): [sign, log|det|, grad[3N], lap].
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T, bool FL>
__global__ __launch_bounds__(64) void k_det(const T *Phi, int64_t B, int K, int n, int TR, int n3, int sp,
                                            double *DR, int rec)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T *LU = (T *)smem_raw;
    T *Mb = LU + n * n;
    int *perm = (int *)(Mb + (FL ? (n3 + 1) * n * n : 0));
    __shared__ int s_sign, s_sing;
    __shared__ double s_log;
    const int lane = threadIdx.x;
    const int64_t wk = blockIdx.x;
    const int64_t w = wk / K;
    const int k = (int)(wk % K);
    if (w >= B) return;
    const int64_t nn = (int64_t)n * n;
    const T *A = Phi + (w * K + k) * TR * nn;
    for (int q = lane; q < n * n; q += 64) LU[q] = A[q];
    for (int q = lane; q < n; q += 64) perm[q] = q;
    if (lane == 0) { s_sign = 1; s_sing = 0; s_log = 0.0; }
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        if (lane == 0) {
            int p = c;
            T best = fabs(LU[c * n + c]);
            for (int r = c + 1; r < n; ++r) {
                T v = fabs(LU[r * n + c]);
                if (v > best) { best = v; p = r; }
            }
            if (best == T(0)) {
                s_sing = 1;
            } else {
                if (p != c) {
                    for (int q = 0; q < n; ++q) { T t = LU[c * n + q]; LU[c * n + q] = LU[p * n + q]; LU[p * n + q] = t; }
                    int t = perm[c]; perm[c] = perm[p]; perm[p] = t;
                    s_sign = -s_sign;
                }
                T piv = LU[c * n + c];
                if (piv < T(0)) s_sign = -s_sign;
                s_log += log((double)fabs(piv));
            }
        }
        __syncthreads();
        if (s_sing) break;
        const T ip = T(1) / LU[c * n + c];
        const int m = n - 1 - c;
        for (int q = lane; q < m; q += 64) LU[(c + 1 + q) * n + c] *= ip;   // multipliers (L below the diagonal)
        __syncthreads();
        for (int q = lane; q < m * m; q += 64) {
            const int r = c + 1 + q / m, cc = c + 1 + q % m;
            LU[r * n + cc] -= LU[r * n + c] * LU[c * n + cc];
        }
        __syncthreads();
    }
    double *out = DR + (w * 2 + sp) * (int64_t)K * rec + (int64_t)k * rec;
    if (s_sing) {
        for (int q = lane; q < rec; q += 64) out[q] = q == 0 ? 0.0 : (q == 1 ? -INFINITY : NAN);
        return;
    }
    if (lane == 0) { out[0] = (double)s_sign; out[1] = s_log; }
    if (!FL) return;
    // solve A M = D for all (3N + 1) right-hand matrices, one column per lane
    const int ncol = (n3 + 1) * n;
    for (int q = lane; q < ncol; q += 64) {
        const int mt = q / n, jj = q % n;
        T *v = Mb + mt * nn;
        const T *D = A + (1 + mt) * nn;
        for (int r = 0; r < n; ++r) v[r * n + jj] = D[perm[r] * n + jj];
        for (int r = 1; r < n; ++r) {
            T acc = v[r * n + jj];
            for (int c = 0; c < r; ++c) acc -= LU[r * n + c] * v[c * n + jj];
            v[r * n + jj] = acc;
        }
        for (int r = n - 1; r >= 0; --r) {
            T acc = v[r * n + jj];
            for (int c = r + 1; c < n; ++c) acc -= LU[r * n + c] * v[c * n + jj];
            v[r * n + jj] = acc / LU[r * n + r];
        }
    }
    __syncthreads();
    double sq = 0.0, trl = 0.0;
    for (int mt = lane; mt <= n3; mt += 64) {
        const T *Mm = Mb + mt * nn;
        T tr = T(0);
        for (int r = 0; r < n; ++r) tr += Mm[r * n + r];
        if (mt < n3) {
            T s2 = T(0);
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c) s2 += Mm[r * n + c] * Mm[c * n + r];
            out[2 + mt] = (double)tr;
            sq += (double)s2;
        } else {
            trl = (double)tr;
        }
    }
    sq = wave_sum(sq);
    trl = wave_sum(trl);
    if (lane == 0) out[2 + n3] = trl - sq;
}

// ---------------------------------------------------------------------------
// forward-Laplacian orbitals, envelope and determinant in one pass: one
// wave64 per (walker, determinant k) of one spin.  The orbital matrix and its
// direction derivatives (Eq. 4 with the product rule) are formed in LDS from
// the head product O and the envelope, never stored to memory:
//   A[i][j]   = a_ij e_ij,           a = orbital value, e = envelope,
//   d_c A     = (d_c a) e + a d_c e  (d_c e nonzero only for c in electron j),
//   lap A     = (lap a) e + a lap e + 2 grad_j a . grad_j e.
// LU with partial pivoting gives sign and log|det A|; the directions are
// solved in chunks of CD (CD n <= 64 columns, one per lane) and reduced to
//   d log|det| / dx_c = tr M_c,  lap log|det| = tr(A^-1 lap A) - sum_c tr(M_c M_c),
// M_c = A^-1 d_c A.  Record per (walker, spin, k): [sign, log|det|, grad[3N], lap].
// Envelope, entries, LU and traces in FP64 for every precision.
// ---------------------------------------------------------------------------
__host__ __device__ inline int orbdet_cd(int n) { return n >= 64 ? 1 : 64 / n; }
constexpr int ORB_PF = 12;   // spins up to this size prefetch a direction's head values

size_t orbdet_lds(int n, bool fl)
{
    const size_t nn = (size_t)n * n;
    return ((fl ? 7 * nn + (size_t)orbdet_cd(n) * nn : nn)) * sizeof(double) + (size_t)n * sizeof(int) + 16;
}
// byte offset of the staged envelope parameters (after the orbdet_lds bytes, 16-byte aligned)
__host__ __device__ inline size_t orbdet_stage_off(int n, bool fl)
{
    const size_t nn = (size_t)n * n;
    return ((fl ? 7 * nn + (size_t)orbdet_cd(n) * nn : nn) * sizeof(double) + (size_t)n * sizeof(int) + 16 + 15) &
           ~(size_t)15;
}

// FL = false: value only (envelope, LU, sign and log|det|), LDS holds the matrix only.
// REG: triangular solves of the directions in registers (spins of 7 ..
// ORB_PF electrons, where LDS, not registers, bounds the resident waves)
// Spins sp0 .. sp0 + nsp - 1 of equal size, B * K workgroups each.
template <typename T, bool FL, bool REG, bool ST>
__global__ __launch_bounds__(64) void k_orbdet(Sys s, const double *x, const T *theta, OrbSpins<T> S, int sp0,
                                               int64_t B, int TR, double *DR, int rec)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int64_t per = B * s.K;
    const int sp = sp0 + (int)(blockIdx.x / per);
    int64_t gof = sp ? S.gof1 : S.gof0, piof = sp ? S.piof1 : S.piof0, sigof = sp ? S.sigof1 : S.sigof0;
    const int64_t ldo = sp ? S.ldo1 : S.ldo0;
    const T *O = sp ? S.O1 : S.O0;
    const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
    const int n3 = 3 * s.N, nn = n * n, CD = orbdet_cd(n);
    double *LU = (double *)smem_raw;      // [n][n] orbitals x electrons, then its LU factors
    double *EV = LU + nn;                 // envelope e
    double *GE = EV + nn;                 // grad_j e [n][n][3]
    double *LE = GE + 3 * nn;             // lap_j e
    double *A0 = LE + nn;                 // orbital value a (with its bias)
    double *Mc = A0 + nn;                 // [CD][n][n] solved directions of one chunk
    int *perm = (int *)(FL ? (double *)(Mc + (size_t)CD * nn) : LU + nn);
    __shared__ int s_sign, s_sing;
    __shared__ double s_log;
    const int lane = threadIdx.x;
    const int64_t wk = blockIdx.x % per;
    const int64_t w = wk / s.K;
    const int k = (int)(wk % s.K);
    if (w >= B) return;

    // ST: this determinant's pi [n][M], Sigma [n][M][1 or 9] and orbital
    // offsets [n] into LDS first (after the matrices and the permutation),
    // requested together instead of once per nucleus
    const T *tp = theta;
    if constexpr (ST) {
        T *prm = reinterpret_cast<T *>(smem_raw + orbdet_stage_off(n, FL));
        const int64_t c0 = (int64_t)k * n, npi = (int64_t)n * s.M, sz = s.iso ? 1 : 9, nsg = npi * sz;
        for (int q = lane; q < npi + nsg + n; q += 64)
            prm[q] = q < npi ? theta[piof + c0 * s.M + q]
                             : (q < npi + nsg ? theta[sigof + c0 * s.M * sz + (q - npi)] : theta[gof + c0 + (q - npi - nsg)]);
        __syncthreads();
        // offsets such that column k n + io lands on staged row io
        tp = prm;
        piof = -c0 * s.M;
        sigof = npi - c0 * s.M * sz;
        gof = npi + nsg - c0;
    }
    // envelope and orbital value of every (orbital io, electron jj)
    for (int q = lane; q < nn; q += 64) {
        const int io = q / n, jj = q - io * n;
        const int col = k * n + io, j = j0 + jj;
        const double *xj = x + (w * s.N + j) * 3;
        double env = 0.0, ge[3] = {0.0, 0.0, 0.0}, le = 0.0;
        for (int m = 0; m < s.M; ++m) env_add<T, FL>(s, tp, piof, sigof, col, m, xj, env, ge, le);
        const double a0 = (double)O[((w * n + jj) * TR) * ldo + col] + (double)tp[gof + col];
        if constexpr (FL) {
            EV[q] = env;
            GE[3 * q] = ge[0]; GE[3 * q + 1] = ge[1]; GE[3 * q + 2] = ge[2];
            LE[q] = le;
            A0[q] = a0;
        }
        LU[q] = a0 * env;
    }
    for (int q = lane; q < n; q += 64) perm[q] = q;
    if (lane == 0) { s_sign = 1; s_sing = 0; s_log = 0.0; }
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        if (lane == 0) {
            int p = c;
            double best = fabs(LU[c * n + c]);
            for (int r = c + 1; r < n; ++r) {
                const double v = fabs(LU[r * n + c]);
                if (v > best) { best = v; p = r; }
            }
            if (best == 0.0) {
                s_sing = 1;
            } else {
                if (p != c) {
                    for (int q = 0; q < n; ++q) { double t = LU[c * n + q]; LU[c * n + q] = LU[p * n + q]; LU[p * n + q] = t; }
                    int t = perm[c]; perm[c] = perm[p]; perm[p] = t;
                    s_sign = -s_sign;
                }
                const double piv = LU[c * n + c];
                if (piv < 0.0) s_sign = -s_sign;
                s_log += log(fabs(piv));
            }
        }
        __syncthreads();
        if (s_sing) break;
        const double ip = 1.0 / LU[c * n + c];
        const int m = n - 1 - c;
        for (int q = lane; q < m; q += 64) LU[(c + 1 + q) * n + c] *= ip;
        __syncthreads();
        for (int q = lane; q < m * m; q += 64) {
            const int r = c + 1 + q / m, cc = c + 1 + q % m;
            LU[r * n + cc] -= LU[r * n + c] * LU[c * n + cc];
        }
        __syncthreads();
    }
    double *out = DR + (w * 2 + sp) * (int64_t)s.K * rec + (int64_t)k * rec;
    if (s_sing) {
        for (int q = lane; q < rec; q += 64) out[q] = q == 0 ? 0.0 : (q == 1 ? -INFINITY : NAN);
        return;
    }
    if (lane == 0) { out[0] = (double)s_sign; out[1] = s_log; }
    if constexpr (!FL) return;

    double sq = 0.0, trl = 0.0;
    for (int t0 = 0; t0 <= n3; t0 += CD) {
        const int nd = n3 + 1 - t0 < CD ? n3 + 1 - t0 : CD;
        // one column (direction d, electron jj) per lane: right-hand side
        // D[perm[r]][jj], then the unit-lower and upper triangular solves
        for (int q = lane; q < nd * n; q += 64) {
            const int d = q / n, jj = q - d * n;
            const int mt = t0 + d, j = j0 + jj;
            const T *Oj = O + ((w * n + jj) * TR) * ldo + k * n;
            double *v = Mc + d * nn;
            if (n <= ORB_PF) {
                // every row's head value is requested before the first is used
                // (the stores below would otherwise order each load after the
                // previous row's store)
                const int orow = mt < n3 ? 1 + mt : n3 + 1;
                int pv[ORB_PF];
                double ov[ORB_PF];
                // rows past n repeat row n - 1: unconditional loads, no branches
#pragma unroll
                for (int r = 0; r < ORB_PF; ++r) pv[r] = perm[r < n ? r : n - 1];
#pragma unroll
                for (int r = 0; r < ORB_PF; ++r) ov[r] = (double)Oj[orow * ldo + pv[r]];
                // REG: right-hand side and both triangular solves in registers
                // (static indices), the solved column stored once; otherwise
                // the right-hand side goes to LDS for the solves below
                double vv[ORB_PF];
#pragma unroll
                for (int r = 0; r < ORB_PF; ++r) {
                    vv[r] = 0.0;
                    if (r < n) {
                        const int io = pv[r], e = io * n + jj;
                        double dv;
                        if (mt < n3) {
                            dv = EV[e] * ov[r];
                            if (mt / 3 == j) dv += A0[e] * GE[3 * e + mt % 3];
                        } else {
                            dv = EV[e] * ov[r] + A0[e] * LE[e];
                            for (int a = 0; a < 3; ++a)
                                dv += 2.0 * (double)Oj[(1 + 3 * j + a) * ldo + io] * GE[3 * e + a];
                        }
                        if constexpr (REG) vv[r] = dv;
                        else v[r * n + jj] = dv;
                    }
                }
                if constexpr (REG) {
#pragma unroll
                for (int r = 1; r < ORB_PF; ++r) {
                    if (r < n) {
                        double acc = vv[r];
#pragma unroll
                        for (int c = 0; c < r; ++c) acc -= LU[r * n + c] * vv[c];
                        vv[r] = acc;
                    }
                }
#pragma unroll
                for (int r = ORB_PF - 1; r >= 0; --r) {
                    if (r < n) {
                        double acc = vv[r];
#pragma unroll
                        for (int c = r + 1; c < ORB_PF; ++c)
                            if (c < n) acc -= LU[r * n + c] * vv[c];
                        vv[r] = acc / LU[r * n + r];
                    }
                }
#pragma unroll
                for (int r = 0; r < ORB_PF; ++r)
                    if (r < n) v[r * n + jj] = vv[r];
                }
            } else {
                for (int r = 0; r < n; ++r) {
                    const int io = perm[r], e = io * n + jj;
                    double dv;
                    if (mt < n3) {
                        dv = EV[e] * (double)Oj[(1 + mt) * ldo + io];
                        if (mt / 3 == j) dv += A0[e] * GE[3 * e + mt % 3];
                    } else {
                        dv = EV[e] * (double)Oj[(n3 + 1) * ldo + io] + A0[e] * LE[e];
                        for (int a = 0; a < 3; ++a) dv += 2.0 * (double)Oj[(1 + 3 * j + a) * ldo + io] * GE[3 * e + a];
                    }
                    v[r * n + jj] = dv;
                }
            }
            if (!REG || n > ORB_PF) {
                for (int r = 1; r < n; ++r) {
                    double acc = v[r * n + jj];
                    for (int c = 0; c < r; ++c) acc -= LU[r * n + c] * v[c * n + jj];
                    v[r * n + jj] = acc;
                }
                for (int r = n - 1; r >= 0; --r) {
                    double acc = v[r * n + jj];
                    for (int c = r + 1; c < n; ++c) acc -= LU[r * n + c] * v[c * n + jj];
                    v[r * n + jj] = acc / LU[r * n + r];
                }
            }
        }
        __syncthreads();
        // tr(M_c M_c) of the tangent directions, tr M of every direction
        for (int q = lane; q < nd * nn; q += 64) {
            const int d = q / nn, rest = q - d * nn;
            if (t0 + d >= n3) continue;
            const int r = rest / n, c = rest - r * n;
            sq += Mc[d * nn + r * n + c] * Mc[d * nn + c * n + r];
        }
        if (lane < nd) {
            double tr = 0.0;
            for (int r = 0; r < n; ++r) tr += Mc[lane * nn + r * n + r];
            if (t0 + lane < n3) out[2 + t0 + lane] = tr;
            else trl = tr;
        }
        __syncthreads();
    }
    sq = wave_sum(sq);
    trl = wave_sum(trl);
    if (lane == 0) out[2 + n3] = trl - sq;
}

// Entries of one small determinant (NS x NS; rows = orbitals io, columns =
// electrons j0 + jj of one spin) for walker w, determinant k: envelope e
// (Eq. 4) and, with FL, its electron-j gradient and Laplacian, the orbital
// value a (head output plus bias) and A = a e; all FP64.
template <typename T, int NS, bool FL>
__device__ __forceinline__ void small_entry(const Sys &s, const double *x, const T *theta, int64_t gof, int64_t piof,
                                            int64_t sigof, const T *O, int64_t ldo, int TR, int j0, int64_t w, int k,
                                            int io, int jj, double &ev, double (&ge)[3], double &le, double &a0,
                                            double &A)
{
    const int col = k * NS + io, j = j0 + jj;
    const double *xj = x + (w * s.N + j) * 3;
    double env = 0.0, g3[3] = {0.0, 0.0, 0.0}, lp = 0.0;
    for (int m = 0; m < s.M; ++m) env_add<T, FL>(s, theta, piof, sigof, col, m, xj, env, g3, lp);
    ev = env;
    ge[0] = g3[0]; ge[1] = g3[1]; ge[2] = g3[2];
    le = lp;
    a0 = (double)O[((w * NS + jj) * TR) * ldo + col] + (double)theta[gof + col];
    A = a0 * env;
}

template <typename T, int NS, bool FL>
__device__ __forceinline__ void small_entries(const Sys &s, const double *x, const T *theta, int64_t gof, int64_t piof,
                                              int64_t sigof, const T *O, int64_t ldo, int TR, int j0, int64_t w, int k,
                                              double (&ev)[NS][NS], double (&ge)[NS][NS][3], double (&le)[NS][NS],
                                              double (&a0)[NS][NS], double (&A)[NS][NS])
{
#pragma unroll
    for (int io = 0; io < NS; ++io)
#pragma unroll
        for (int jj = 0; jj < NS; ++jj)
            small_entry<T, NS, FL>(s, x, theta, gof, piof, sigof, O, ldo, TR, j0, w, k, io, jj, ev[io][jj], ge[io][jj],
                                   le[io][jj], a0[io][jj], A[io][jj]);
}

// LU with partial pivoting of A in place (rows = orbitals): row permutation,
// sign and log|det A|; sing when a pivot column is zero.
template <int NS>
__device__ __forceinline__ void small_lu(double (&A)[NS][NS], int (&perm)[NS], int &sgn, double &lg, bool &sing)
{
#pragma unroll
    for (int r = 0; r < NS; ++r) perm[r] = r;
    sgn = 1;
    lg = 0.0;
    sing = false;
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        int p = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < NS; ++r)
            if (fabs(A[r][c]) > best) { best = fabs(A[r][c]); p = r; }
        if (best == 0.0) { sing = true; break; }
        if (p != c) {
#pragma unroll
            for (int r = c + 1; r < NS; ++r)
                if (r == p) {
#pragma unroll
                    for (int q = 0; q < NS; ++q) { const double t = A[c][q]; A[c][q] = A[r][q]; A[r][q] = t; }
                    const int t = perm[c]; perm[c] = perm[r]; perm[r] = t;
                }
            sgn = -sgn;
        }
        const double piv = A[c][c];
        if (piv < 0.0) sgn = -sgn;
        lg += log(fabs(piv));
        const double ip = 1.0 / piv;
#pragma unroll
        for (int r = c + 1; r < NS; ++r) {
            A[r][c] *= ip;
#pragma unroll
            for (int q = c + 1; q < NS; ++q) A[r][q] -= A[r][c] * A[c][q];
        }
    }
}

// Small spins: one thread per (walker, determinant k) with the
// matrices in registers (two adjacent threads in the forward-Laplacian form,
// each taking half of the directions; four measured slower).  Same quantities as k_orbdet; here
// the directions use the explicit inverse from the pivoted LU,
// M_c = A^-1 d_c A.  The spin's envelope parameters and orbital offsets are
// copied into LDS once per workgroup (when they fit: SMALL_STAGE_MAX
// elements), and the orbital rows a thread reads are requested before the
// envelope arithmetic, SMALL_DIRS directions at a time, so that a thread
// waits for global memory about twice instead of once per direction.
constexpr int SMALL_DIRS = 8;
constexpr int SMALL_STAGE_MAX = 8192;

// elements of the staged parameter block of one spin: pi [K n][M], Sigma
// [K n][M][1 or 9], orbital offsets g [K n]
inline __host__ __device__ int64_t small_stage_elems(const Sys &s, int n)
{
    const int64_t kn = (int64_t)s.K * n;
    return kn * s.M * (s.iso ? 2 : 10) + kn;
}

template <typename T, int NS, bool FL, bool ST>
__global__ __launch_bounds__(256) void k_orbdet_small(Sys s, const double *x, const T *theta, OrbSpins<T> S, int sp0,
                                                      int64_t B, int TR, double *DR, int rec)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char small_smem[];
    // spins sp0 .. of NS electrons each, ceil(H B K / 256) workgroups per spin
    constexpr int H = FL ? 2 : 1;                         // threads per determinant
    const int64_t per = B * s.K * H, gsp = (per + 255) / 256;
    const int sp = sp0 + (int)(blockIdx.x / gsp);
    int64_t gof = sp ? S.gof1 : S.gof0, piof = sp ? S.piof1 : S.piof0, sigof = sp ? S.sigof1 : S.sigof0;
    const int64_t ldo = sp ? S.ldo1 : S.ldo0;
    const T *O = sp ? S.O1 : S.O0;
    const int j0 = sp == 0 ? 0 : s.nu;
    const int n3 = 3 * s.N;
    const int64_t tid = (blockIdx.x % gsp) * (int64_t)blockDim.x + threadIdx.x;
    // the spin's parameters into LDS (ST: they fit; every thread of the
    // workgroup takes part before any of them leaves)
    const T *tp = theta;
    if constexpr (ST) {
        const int64_t nst = small_stage_elems(s, NS);
        T *sm = reinterpret_cast<T *>(small_smem);
        const int64_t kn = (int64_t)s.K * NS, npi = kn * s.M, nsg = npi * (s.iso ? 1 : 9);
        for (int64_t q = threadIdx.x; q < nst; q += blockDim.x)
            sm[q] = q < npi ? theta[piof + q] : (q < npi + nsg ? theta[sigof + (q - npi)] : theta[gof + (q - npi - nsg)]);
        __syncthreads();
        tp = sm;
        piof = 0;
        sigof = npi;
        gof = npi + nsg;
    }
    // the H threads of a determinant are adjacent lanes (per is a multiple of
    // H, so either all of them return here or none)
    if (tid >= per) return;
    const int hh = (int)(tid % H);
    const int64_t id = tid / H;
    const int64_t w = id / s.K;
    const int k = (int)(id % s.K);
    // directions mt0 .. mt1 - 1 of the 3N tangents and the Laplacian (mt = 3N);
    // direction mt reads orbital row 1 + mt (the Laplacian row is 3N + 1), the
    // Laplacian also electron j's own tangent rows
    const int mt0 = hh * ((n3 + 1) / H), mt1 = hh + 1 == H ? n3 + 1 : (hh + 1) * ((n3 + 1) / H);
    const T *Ob = O + (w * NS * TR) * ldo + k * NS;      // row (jj, t) at (jj TR + t) ldo
    T ov[SMALL_DIRS][NS][NS], lj[NS][NS][3];
    auto load_dirs = [&](int mb) {
#pragma unroll
        for (int u = 0; u < SMALL_DIRS; ++u)
#pragma unroll
            for (int io = 0; io < NS; ++io)
#pragma unroll
                for (int jj = 0; jj < NS; ++jj)
                    ov[u][io][jj] = mb + u < mt1 ? Ob[((int64_t)jj * TR + 1 + mb + u) * ldo + io] : T(0);
    };
    if constexpr (FL) {
        load_dirs(mt0);
#pragma unroll
        for (int io = 0; io < NS; ++io)
#pragma unroll
            for (int jj = 0; jj < NS; ++jj)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    lj[io][jj][a] = mt1 == n3 + 1 ? Ob[((int64_t)jj * TR + 1 + 3 * (j0 + jj) + a) * ldo + io] : T(0);
    }
    double ev[NS][NS], ge[NS][NS][3], le[NS][NS], a0[NS][NS], A[NS][NS];
    if constexpr (H == 2 && NS == 2) {
        // each of the two threads forms one orbital row (io = hh), then the
        // pair swaps them (adjacent lanes)
        double rv[NS][7];                                 // per electron: e, grad e (3), lap e, a, A
#pragma unroll
        for (int jj = 0; jj < NS; ++jj) {
            double g3[3];
            small_entry<T, NS, FL>(s, x, tp, gof, piof, sigof, O, ldo, TR, j0, w, k, hh, jj, rv[jj][0], g3, rv[jj][4],
                                   rv[jj][5], rv[jj][6]);
            rv[jj][1] = g3[0]; rv[jj][2] = g3[1]; rv[jj][3] = g3[2];
        }
#pragma unroll
        for (int jj = 0; jj < NS; ++jj) {
            double ov7[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) ov7[q] = __shfl_xor(rv[jj][q], 1);
#pragma unroll
            for (int io = 0; io < NS; ++io) {
                ev[io][jj] = io == hh ? rv[jj][0] : ov7[0];
                ge[io][jj][0] = io == hh ? rv[jj][1] : ov7[1];
                ge[io][jj][1] = io == hh ? rv[jj][2] : ov7[2];
                ge[io][jj][2] = io == hh ? rv[jj][3] : ov7[3];
                le[io][jj] = io == hh ? rv[jj][4] : ov7[4];
                a0[io][jj] = io == hh ? rv[jj][5] : ov7[5];
                A[io][jj] = io == hh ? rv[jj][6] : ov7[6];
            }
        }
    } else {
        small_entries<T, NS, FL>(s, x, tp, gof, piof, sigof, O, ldo, TR, j0, w, k, ev, ge, le, a0, A);
    }
    // LU with partial pivoting (rows = orbitals), then the inverse
    int perm[NS], sgn;
    double lg;
    bool sing;
    small_lu<NS>(A, perm, sgn, lg, sing);
    double *out = DR + (w * 2 + sp) * (int64_t)s.K * rec + (int64_t)k * rec;
    if (sing) {
        if (hh == 0) {
            out[0] = 0.0;
            out[1] = -INFINITY;
            for (int q = 2; q < rec; ++q) out[q] = NAN;
        }
        return;
    }
    if (hh == 0) {
        out[0] = (double)sgn;
        out[1] = lg;
    }
    if constexpr (!FL) return;
    // inverse: column e of A^-1 solves (LU) y = P e_e
    double Ai[NS][NS];
#pragma unroll
    for (int e = 0; e < NS; ++e) {
        double v[NS];
#pragma unroll
        for (int r = 0; r < NS; ++r) v[r] = perm[r] == e ? 1.0 : 0.0;
#pragma unroll
        for (int r = 1; r < NS; ++r)
#pragma unroll
            for (int c = 0; c < r; ++c) v[r] -= A[r][c] * v[c];
#pragma unroll
        for (int r = NS - 1; r >= 0; --r) {
#pragma unroll
            for (int c = r + 1; c < NS; ++c) v[r] -= A[r][c] * v[c];
            v[r] /= A[r][r];
        }
#pragma unroll
        for (int r = 0; r < NS; ++r) Ai[r][e] = v[r];
    }
    // directions: D = d_c A (tangents) or lap A; M = A^-1 D
    double sq = 0.0, trl = 0.0;
    for (int mb = mt0; mb < mt1; mb += SMALL_DIRS) {
        if (mb != mt0) load_dirs(mb);
#pragma unroll
        for (int u = 0; u < SMALL_DIRS; ++u) {
            const int mt = mb + u;
            if (mt >= mt1) break;
            double D[NS][NS];
#pragma unroll
            for (int io = 0; io < NS; ++io)
#pragma unroll
                for (int jj = 0; jj < NS; ++jj) {
                    const int j = j0 + jj;
                    double dv;
                    if (mt < n3) {
                        dv = ev[io][jj] * (double)ov[u][io][jj];
                        if (mt / 3 == j) dv += a0[io][jj] * ge[io][jj][mt % 3];
                    } else {
                        dv = ev[io][jj] * (double)ov[u][io][jj] + a0[io][jj] * le[io][jj];
                        for (int a = 0; a < 3; ++a) dv += 2.0 * (double)lj[io][jj][a] * ge[io][jj][a];
                    }
                    D[io][jj] = dv;
                }
            double M[NS][NS];
#pragma unroll
            for (int i = 0; i < NS; ++i)
#pragma unroll
                for (int c = 0; c < NS; ++c) {
                    double acc = 0.0;
#pragma unroll
                    for (int r = 0; r < NS; ++r) acc += Ai[i][r] * D[r][c];
                    M[i][c] = acc;
                }
            double tr = 0.0;
#pragma unroll
            for (int i = 0; i < NS; ++i) tr += M[i][i];
            if (mt < n3) {
                out[2 + mt] = tr;
#pragma unroll
                for (int i = 0; i < NS; ++i)
#pragma unroll
                    for (int c = 0; c < NS; ++c) sq += M[i][c] * M[c][i];
            } else {
                trl = tr;
            }
        }
    }
    // the H threads' sums of tr(M_c^2) added in thread order; the Laplacian
    // direction is the last thread's
    const int l0 = (int)(threadIdx.x & 63) - hh;
    double sqt = __shfl(sq, l0, 64);
#pragma unroll
    for (int q = 1; q < H; ++q) sqt += __shfl(sq, l0 + q, 64);
    if (hh == H - 1) out[2 + n3] = trl - sqt;
}

// ---------------------------------------------------------------------------
// per walker, FP64: psi = sum_k s_k exp(l_k), l_k = l_k_up + l_k_dn;
// log|psi| = l_max + log|sum_k s_k exp(l_k - l_max)|, weights
// w_k = s_k exp(l_k - l_max) / sum; E_kin = -1/2 (lap psi)/psi
// = -1/2 sum_k w_k (lap l_k + |grad l_k|^2)  (Eq. 3 summed over coordinates);
// Coulomb sums of Eq. 2 with wavefront reductions.
// ---------------------------------------------------------------------------
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <bool FL>
__global__ __launch_bounds__(64) void k_combine(Sys s, const double *x, const double *DR, int rec, int64_t B,
                                                double vnn, double *log_abs, int8_t *sign, double *e_loc,
                                                double *parts, AcceptArgs acc)
{
    __shared__ double s_w[FN_MAX_DET];
    const int lane = threadIdx.x;
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int K = s.K, n3 = 3 * s.N;
    const double *ru = DR + (w * 2 + 0) * (int64_t)K * rec;
    const double *rd = DR + (w * 2 + 1) * (int64_t)K * rec;
    double sk = 0.0, lk = -INFINITY;
    if (lane < K) {
        double su = s.nu > 0 ? ru[lane * rec] : 1.0, sd = s.nd > 0 ? rd[lane * rec] : 1.0;
        double lu = s.nu > 0 ? ru[lane * rec + 1] : 0.0, ld = s.nd > 0 ? rd[lane * rec + 1] : 0.0;
        sk = su * sd;
        lk = sk != 0.0 ? lu + ld : -INFINITY;
    }
    const double lmax = wave_max(lk);
    double ek = (lane < K && sk != 0.0) ? sk * exp(lk - lmax) : 0.0;
    const double S = wave_sum(ek);
    const bool node = !(lmax > -INFINITY) || S == 0.0 || !(S == S);
    const double lpsi = node ? -INFINITY : lmax + log(fabs(S));
    if (lane == 0) {
        if (log_abs) log_abs[w] = lpsi;
        if (sign) sign[w] = node ? 0 : (S > 0 ? 1 : -1);
    }
    if constexpr (!FL) {
        if (acc.x) {
            // the acceptance rule of the Metropolis step for this walker's proposal
            const bool take = isfinite(lpsi) && log(acc.u[w]) <= 2.0 * (lpsi - acc.log_abs[w]);
            if (take) {
                for (int q = lane; q < n3; q += 64) acc.x[w * n3 + q] = acc.xp[w * n3 + q];
                if (lane == 0) {
                    acc.log_abs[w] = lpsi;
                    if (acc.n_accept) acc.n_accept[w] += 1;
                }
            }
        }
        return;
    }
    if (lane < K) s_w[lane] = node ? 0.0 : ek / S;
    __syncthreads();
    // sum_k w_k |grad l_k|^2 over coordinates, and sum_k w_k lap l_k (one
    // item per (determinant, coordinate): a lane's loads are independent)
    double q = 0.0;
    for (int it = lane; it < K * n3; it += 64) {
        const int k = it / n3, c = it - k * n3;
        const double gu = s.nu > 0 ? ru[k * rec + 2 + c] : 0.0, gd = s.nd > 0 ? rd[k * rec + 2 + c] : 0.0;
        const double g = gu + gd;
        q += s_w[k] * g * g;
    }
    double lsum = 0.0;
    if (lane < K) {
        double lu = s.nu > 0 ? ru[lane * rec + 2 + n3] : 0.0, ld = s.nd > 0 ? rd[lane * rec + 2 + n3] : 0.0;
        lsum = s_w[lane] * (lu + ld);
    }
    q = wave_sum(q);
    lsum = wave_sum(lsum);
    const double kin = node ? NAN : -0.5 * (lsum + q);
    // Coulomb: electron pairs and electron-nucleus pairs over the lanes
    const double *xw = x + w * n3;
    double vee = 0.0, ven = 0.0;
    const int npair = s.N * (s.N - 1) / 2;
    for (int p = lane; p < npair; p += 64) {
        int i = 0, rem = p;
        while (rem >= s.N - 1 - i) { rem -= s.N - 1 - i; ++i; }
        int j = i + 1 + rem;
        double d0 = xw[3 * i] - xw[3 * j], d1 = xw[3 * i + 1] - xw[3 * j + 1], d2 = xw[3 * i + 2] - xw[3 * j + 2];
        vee += 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    for (int p = lane; p < s.N * s.M; p += 64) {
        int i = p / s.M, m = p % s.M;
        double d0 = xw[3 * i] - s.R[m][0], d1 = xw[3 * i + 1] - s.R[m][1], d2 = xw[3 * i + 2] - s.R[m][2];
        ven -= s.Z[m] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    vee = wave_sum(vee);
    ven = wave_sum(ven);
    if (lane == 0) {
        e_loc[w] = kin + vee + ven + vnn;
        if (parts) {
            parts[4 * w] = kin; parts[4 * w + 1] = vee; parts[4 * w + 2] = ven; parts[4 * w + 3] = vnn;
        }
    }
}

// Value form, both spins of NS electrons, K <= 32 determinants: the orbital
// / determinant stage and the combine in one launch.  A group of G lanes
// (G = 32 when 2K <= 32, else 64) takes one walker; lane sp K + k forms
// determinant k of spin sp as k_orbdet_small does.  Lanes k < K then pair
// the spins and reduce over k with the butterflies of k_combine in the same
// order (that kernel's first step only adds lanes without a determinant), so
// log|psi|, its sign and the Metropolis decision are those of the two
// separate kernels.
template <typename T, int NS, int G>
__global__ __launch_bounds__(256) void k_orbdet_combine(Sys s, const double *x, const T *theta, OrbSpins<T> S,
                                                        int64_t B, int TR, double *log_abs, int8_t *sign,
                                                        AcceptArgs acc)
{
    const int lane = threadIdx.x & 63, gl = lane & (G - 1);
    const int64_t w = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    const int K = s.K, n3 = 3 * s.N;
    const bool wok = w < B;
    double sg = 0.0, lg = -INFINITY;              // lanes without a determinant
    if (wok && gl < 2 * K) {
        const int sp = gl < K ? 0 : 1, k = gl < K ? gl : gl - K;
        const int64_t gof = sp ? S.gof1 : S.gof0, piof = sp ? S.piof1 : S.piof0, sigof = sp ? S.sigof1 : S.sigof0;
        const int64_t ldo = sp ? S.ldo1 : S.ldo0;
        const T *O = sp ? S.O1 : S.O0;
        double ev[NS][NS], ge[NS][NS][3], le[NS][NS], a0[NS][NS], A[NS][NS];
        small_entries<T, NS, false>(s, x, theta, gof, piof, sigof, O, ldo, TR, sp ? s.nu : 0, w, k, ev, ge, le, a0, A);
        int perm[NS], sgn;
        double l;
        bool sing;
        small_lu<NS>(A, perm, sgn, l, sing);
        sg = sing ? 0.0 : (double)sgn;
        lg = sing ? -INFINITY : l;
    }
    // spin-down determinant k from lane K + k of the group
    const int src = gl < K ? lane + K : lane;
    const double sd = __shfl(sg, src, 64), ld = __shfl(lg, src, 64);
    double sk = 0.0, lk = -INFINITY;
    if (gl < K) {
        sk = sg * sd;
        lk = sk != 0.0 ? lg + ld : -INFINITY;
    }
    double lmax = lk;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off, 64));
    double sum = (gl < K && sk != 0.0) ? sk * exp(lk - lmax) : 0.0;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    const bool node = !(lmax > -INFINITY) || sum == 0.0 || !(sum == sum);
    const double lpsi = node ? -INFINITY : lmax + log(fabs(sum));
    if (!wok) return;
    if (gl == 0) {
        if (log_abs) log_abs[w] = lpsi;
        if (sign) sign[w] = node ? 0 : (sum > 0 ? 1 : -1);
    }
    if (acc.x) {
        const bool take = isfinite(lpsi) && log(acc.u[w]) <= 2.0 * (lpsi - acc.log_abs[w]);
        if (take) {
            for (int q = gl; q < n3; q += G) acc.x[w * n3 + q] = acc.xp[w * n3 + q];
            if (gl == 0) {
                acc.log_abs[w] = lpsi;
                if (acc.n_accept) acc.n_accept[w] += 1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n, int bs = 256)
{
    int64_t g = (n + bs - 1) / bs;
    if (g > 1 << 20) g = 1 << 20;
    if (g < 1) g = 1;
    return (unsigned)g;
}

template <typename T>
void launch_pack(const T *theta, const PackList &pl, hipStream_t st)
{
    if (pl.n <= 0) return;
    PackList q = pl;
    int64_t nb = 0;
    for (int k = 0; k < q.n; ++k) {
        q.seg[k].bbegin = (int)nb;
        nb += (q.seg[k].count + 255) / 256;
    }
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_pack<T>, dim3((unsigned)nb), dim3(256), 0, st, theta, q);
}

template <typename T>
void launch_features(const Sys &s, const double *x, int64_t B, int TR, int HW0, int64_t ldh, T *H, T *G,
                     hipStream_t st)
{
    const int64_t live = TR == 1 ? 1 : 3 * s.N + 2;
    const int64_t items = B * s.N * TR * (HW0 / 4) + (G ? B * live * 2 * (HW0 / 4) : 0);
    hipLaunchKernelGGL(k_features<T>, dim3(grid_for(items)), dim3(256), 0, st, s, x, B, TR, HW0, ldh, H, G);
}

// LDS of a pair-stream workgroup holding WB (walker, electron) rows
static size_t pair_stream_lds_wb(const Sys &s, bool fl, size_t elem, int WB)
{
    const int w2p = round_up(s.w2, 4), wp = w2p > 4 ? w2p : 4;
    const size_t per = (size_t)s.N * ((fl ? 8 : 1) * wp + 128 / elem);
    return (2 * (size_t)WB * per + (size_t)pair_w_offset(s, s.L > 1 ? s.L - 1 : 0)) * elem;
}

size_t pair_stream_lds(const Sys &s, bool fl, size_t elem) { return pair_stream_lds_wb(s, fl, elem, 1); }

// Output columns per thread (1, 2 or 4) and (walker, electron) rows per
// workgroup: about 256 (pair, column group) items, within 64 KiB of LDS.  The
// forward-Laplacian form takes fewer columns per thread for small N * w2
// (more threads share the LDS rows of a pair); the value form takes 4.
int g_pair_oc = 0, g_pair_items = 0;
int g_det_stage = 1;

static int pair_stream_oc(const Sys &s, bool fl)
{
    if (g_pair_oc) return g_pair_oc;
    if (!fl) return 4;                                    // value rows: fewest LDS reads per product
    const int w2p = round_up(s.w2, 4);
    return s.N * w2p <= 256 ? 1 : (s.N * w2p <= 512 ? 2 : 4);
}

static int pair_stream_wb(const Sys &s, bool fl, size_t elem)
{
    const int target = g_pair_items ? g_pair_items : 256;
    const int items = s.N * (round_up(s.w2, 4) / pair_stream_oc(s, fl));
    int wb = items >= target ? 1 : target / items;
    while (wb > 1 && pair_stream_lds_wb(s, fl, elem, wb) > 64 * 1024) --wb;
    return wb;
}

template <typename T, bool FL>
static void launch_pair_oc(const Sys &s, const double *x, const T *theta, const ParamLayout &P, int64_t B, int TR,
                           int64_t ldg, int64_t gi_layer_stride, int GW0, int GW1, T *GI, hipStream_t st)
{
    const int wb = pair_stream_wb(s, FL, sizeof(T));
    const size_t lds = pair_stream_lds_wb(s, FL, sizeof(T), wb);
    dim3 grid((unsigned)((B * s.N + wb - 1) / wb));
    switch (pair_stream_oc(s, FL)) {
    case 1:
        hipLaunchKernelGGL((k_pair_stream<T, FL, 1>), grid, dim3(256), lds, st, s, x, theta, P, B, TR, ldg,
                           gi_layer_stride, GW0, GW1, wb, GI);
        break;
    case 2:
        hipLaunchKernelGGL((k_pair_stream<T, FL, 2>), grid, dim3(256), lds, st, s, x, theta, P, B, TR, ldg,
                           gi_layer_stride, GW0, GW1, wb, GI);
        break;
    default:
        hipLaunchKernelGGL((k_pair_stream<T, FL, 4>), grid, dim3(256), lds, st, s, x, theta, P, B, TR, ldg,
                           gi_layer_stride, GW0, GW1, wb, GI);
        break;
    }
}

// matrix-core pair kernel: LDS of WB (walker, electron) rows, pair rows per
// workgroup about g_pair_items (default 128 in the forward-Laplacian form,
// 64 in the value form: two or one row blocks per wave) within 64 KiB
bool g_pair_mfma = true;

static size_t pair_mfma_lds_wb(const Sys &s, bool fl, int WB)
{
    const int wc = round_up(s.w2, 16);
    const size_t rows = (size_t)round_up(WB * s.N * (fl ? 8 : 1), 16);
    return (rows * (wc + 4) + (size_t)pair_mfma_woff(s, s.L > 1 ? s.L - 1 : 0)) * sizeof(float);
}

static bool pair_mfma_ok(const Sys &s, bool fl)
{
    return g_pair_mfma && s.w2 <= 64 && s.w2 % 4 == 0 && pair_mfma_lds_wb(s, fl, 1) <= 64 * 1024;
}

static int pair_mfma_wb(const Sys &s, bool fl)
{
    const int rows = s.N * (fl ? 8 : 1);
    const int target = g_pair_items ? g_pair_items : (fl ? 128 : 64);
    int wb = rows >= target ? 1 : target / rows;
    while (wb > 1 && pair_mfma_lds_wb(s, fl, wb) > 64 * 1024) --wb;
    return wb;
}

template <bool FL>
static void launch_pair_mfma(const Sys &s, const double *x, const float *wpair, int64_t B, int TR, int64_t ldg,
                             int64_t gi_layer_stride, int GW0, int GW1, float *GI, hipStream_t st)
{
    const int wb = pair_mfma_wb(s, FL);
    const size_t lds = pair_mfma_lds_wb(s, FL, wb);
    dim3 grid((unsigned)((B * s.N + wb - 1) / wb));
    hipLaunchKernelGGL((k_pair_mfma<FL>), grid, dim3(256), lds, st, s, x, wpair, B, TR, ldg, gi_layer_stride, GW0,
                       GW1, wb, GI);
}

template <typename T>
void launch_pair_stream(const Sys &s, const double *x, const T *theta, const ParamLayout &P, int64_t B, int TR,
                        bool fl, int64_t ldg, int64_t gi_layer_stride, int GW0, int GW1, const float *wpair, T *GI,
                        hipStream_t st)
{
    if constexpr (std::is_same<T, float>::value) {
        if (wpair && pair_mfma_ok(s, fl)) {
            if (fl) launch_pair_mfma<true>(s, x, wpair, B, TR, ldg, gi_layer_stride, GW0, GW1, GI, st);
            else launch_pair_mfma<false>(s, x, wpair, B, TR, ldg, gi_layer_stride, GW0, GW1, GI, st);
            return;
        }
    }
    if (fl)
        launch_pair_oc<T, true>(s, x, theta, P, B, TR, ldg, gi_layer_stride, GW0, GW1, GI, st);
    else
        launch_pair_oc<T, false>(s, x, theta, P, B, TR, ldg, gi_layer_stride, GW0, GW1, GI, st);
}

template <typename T>
void launch_spin_mean(const T *H, int64_t ldh, int64_t B, int N, int nu, int TR, int dh, int HWl, T *G,
                      hipStream_t st)
{
    // rows value .. Laplacian only (the mean-field product reads no padding row)
    const int live = TR == 1 ? 1 : 3 * N + 2;
    const int64_t items = B * live * (sizeof(T) == 4 ? HWl / 2 : 2 * HWl);
    hipLaunchKernelGGL(k_spin_mean<T>, dim3(grid_for(items)), dim3(256), 0, st, H, ldh, B, N, nu, TR, live, dh, HWl,
                       G);
}

template <typename T>
void launch_layer_epi(const T *X, const T *Pw, const T *bias, const T *Hin, T *Hout, int64_t ldh, int64_t B, int N,
                      int TR, int n3, int w1, int W1p, int resid, bool fl, T *Tout, hipStream_t st)
{
    dim3 g((unsigned)(B * N));
    if (fl)
        hipLaunchKernelGGL((k_layer_epi<T, true>), g, dim3(256), 0, st, X, Pw, bias, Hin, Hout, ldh, N, TR, n3, w1,
                           W1p, resid, Tout);
    else
        hipLaunchKernelGGL((k_layer_epi<T, false>), g, dim3(256), 0, st, X, Pw, bias, Hin, Hout, ldh, N, TR, n3, w1,
                           W1p, resid, Tout);
}

template <typename T>
void launch_envelope(const Sys &s, const double *x, const T *theta, int64_t gof, int64_t piof, int64_t sigof, int sp,
                     const T *O, int64_t ldo, int64_t B, int TR, bool fl, double *Phi, hipStream_t st)
{
    int n = sp == 0 ? s.nu : s.nd;
    dim3 g(grid_for(B * n * s.K * n));
    if (fl)
        hipLaunchKernelGGL((k_envelope<T, true>), g, dim3(256), 0, st, s, x, theta, gof, piof, sigof, sp, O, ldo, B,
                           TR, Phi);
    else
        hipLaunchKernelGGL((k_envelope<T, false>), g, dim3(256), 0, st, s, x, theta, gof, piof, sigof, sp, O, ldo, B,
                           TR, Phi);
}

size_t det_lds(int n, int n3, bool fl, size_t elem)
{
    return ((size_t)n * n + (fl ? (size_t)(n3 + 1) * n * n : 0)) * elem + (size_t)n * sizeof(int) + 16;
}

void launch_det(const double *Phi, int64_t B, int K, int n, int TR, int n3, int sp, bool fl, double *DR, int rec,
                hipStream_t st)
{
    typedef double T;
    size_t lds = det_lds(n, n3, fl, sizeof(T));
    dim3 g((unsigned)(B * K));
    if (fl)
        hipLaunchKernelGGL((k_det<T, true>), g, dim3(64), lds, st, Phi, B, K, n, TR, n3, sp, DR, rec);
    else
        hipLaunchKernelGGL((k_det<T, false>), g, dim3(64), lds, st, Phi, B, K, n, TR, n3, sp, DR, rec);
}

template <typename T, int NS, bool FL>
static void launch_small(const Sys &s, const double *x, const T *theta, const OrbSpins<T> &S, int sp0, int nsp,
                         int64_t B, int TR, double *DR, int rec, hipStream_t st)
{
    const int H = FL ? 2 : 1;                             // threads per determinant (as in the kernel)
    const dim3 gs((unsigned)(nsp * ((H * B * s.K + 255) / 256)));
    const int64_t nst = small_stage_elems(s, NS);
    if (g_det_stage && nst <= SMALL_STAGE_MAX)
        hipLaunchKernelGGL((k_orbdet_small<T, NS, FL, true>), gs, dim3(256), (size_t)nst * sizeof(T), st, s, x, theta, S,
                           sp0, B, TR, DR, rec);
    else
        hipLaunchKernelGGL((k_orbdet_small<T, NS, FL, false>), gs, dim3(256), 0, st, s, x, theta, S, sp0, B, TR, DR, rec);
}

// spins sp0 .. sp0 + nsp - 1 (of n electrons each) in one launch: one thread
// per determinant where its matrices fit in registers (n <= 2 in
// forward-Laplacian form, n <= 8 for the value alone), one wave otherwise
template <typename T, bool FL>
static void launch_orbdet_spins(const Sys &s, const double *x, const T *theta, const OrbSpins<T> &S, int sp0, int nsp,
                                int n, int64_t B, int TR, double *DR, int rec, hipStream_t st)
{
#define FN_SMALL(NS)                                                                                        \
    case NS: launch_small<T, NS, FL>(s, x, theta, S, sp0, nsp, B, TR, DR, rec, st); return;
    switch (n) {
        FN_SMALL(1)
        FN_SMALL(2)
    default: break;
    }
    if constexpr (!FL) {
        switch (n) {
            FN_SMALL(3)
            FN_SMALL(4)
            FN_SMALL(5)
            FN_SMALL(6)
            FN_SMALL(7)
            FN_SMALL(8)
        default: break;
        }
    }
#undef FN_SMALL
    const dim3 g((unsigned)(nsp * B * s.K));
    // the determinant's envelope parameters staged in LDS when that adds at
    // most a quarter to the workgroup's LDS (more lowers the resident
    // workgroups by more than the staging saves: H20, 20 nuclei, 46%
    // slower; LiF, 2 nuclei, 8% faster)
    const size_t base = orbdet_lds(n, FL);
    const size_t staged = orbdet_stage_off(n, FL) + ((size_t)n * s.M * (s.iso ? 2 : 10) + n) * sizeof(T);
    const bool st_ok = g_det_stage && 4 * (staged - base) <= base && staged <= 64 * 1024;
    if constexpr (FL) {
        if (n >= 7 && n <= ORB_PF) {
            if (st_ok)
                hipLaunchKernelGGL((k_orbdet<T, true, true, true>), g, dim3(64), staged, st, s, x, theta, S, sp0,
                                   B, TR, DR, rec);
            else
                hipLaunchKernelGGL((k_orbdet<T, true, true, false>), g, dim3(64), base, st, s, x, theta, S, sp0, B, TR,
                                   DR, rec);
            return;
        }
    }
    if (st_ok)
        hipLaunchKernelGGL((k_orbdet<T, FL, false, true>), g, dim3(64), staged, st, s, x, theta, S, sp0, B, TR,
                           DR, rec);
    else
        hipLaunchKernelGGL((k_orbdet<T, FL, false, false>), g, dim3(64), base, st, s, x, theta, S, sp0, B, TR, DR,
                           rec);
}

template <typename T>
void launch_orbdet(const Sys &s, const double *x, const T *theta, const OrbSpins<T> &S, int64_t B, int TR, bool fl,
                   double *DR, int rec, hipStream_t st)
{
    auto run = [&](int sp0, int nsp, int n) {
        if (fl) launch_orbdet_spins<T, true>(s, x, theta, S, sp0, nsp, n, B, TR, DR, rec, st);
        else launch_orbdet_spins<T, false>(s, x, theta, S, sp0, nsp, n, B, TR, DR, rec, st);
    };
    if (s.nu > 0 && s.nu == s.nd) {
        run(0, 2, s.nu);
        return;
    }
    if (s.nu > 0) run(0, 1, s.nu);
    if (s.nd > 0) run(1, 1, s.nd);
}

template <typename T>
bool launch_orbdet_combine(const Sys &s, const double *x, const T *theta, const OrbSpins<T> &S, int64_t B, int TR,
                           double *log_abs, int8_t *sign, const AcceptArgs &acc, hipStream_t st)
{
    if (s.nu != s.nd || s.nu < 1 || s.nu > 8 || s.K > 32 || B <= 0) return false;
    const bool g32 = 2 * s.K <= 32;
    const dim3 g((unsigned)((B + (g32 ? 8 : 4) - 1) / (g32 ? 8 : 4)));
#define FN_OC(NS)                                                                                                  \
    case NS:                                                                                                       \
        if (g32) hipLaunchKernelGGL((k_orbdet_combine<T, NS, 32>), g, dim3(256), 0, st, s, x, theta, S, B, TR,     \
                                    log_abs, sign, acc);                                                           \
        else hipLaunchKernelGGL((k_orbdet_combine<T, NS, 64>), g, dim3(256), 0, st, s, x, theta, S, B, TR,         \
                                log_abs, sign, acc);                                                               \
        return true;
    switch (s.nu) {
        FN_OC(1) FN_OC(2) FN_OC(3) FN_OC(4) FN_OC(5) FN_OC(6) FN_OC(7) FN_OC(8)
    default: return false;
    }
#undef FN_OC
}

void launch_combine(const Sys &s, const double *x, const double *DR, int rec, int64_t B, double vnn, double *log_abs,
                    int8_t *sign, double *e_loc, double *parts, bool fl, const AcceptArgs &acc, hipStream_t st)
{
    if (fl)
        hipLaunchKernelGGL(k_combine<true>, dim3((unsigned)B), dim3(64), 0, st, s, x, DR, rec, B, vnn, log_abs, sign,
                           e_loc, parts, AcceptArgs{});
    else
        hipLaunchKernelGGL(k_combine<false>, dim3((unsigned)B), dim3(64), 0, st, s, x, DR, rec, B, vnn, log_abs, sign,
                           e_loc, parts, acc);
}

#define FN_INST(T)                                                                                                  \
    template void launch_pack<T>(const T *, const PackList &, hipStream_t);                                          \
    template void launch_features<T>(const Sys &, const double *, int64_t, int, int, int64_t, T *, T *,             \
                                     hipStream_t);                                                                  \
    template void launch_pair_stream<T>(const Sys &, const double *, const T *, const ParamLayout &, int64_t, int,   \
                                        bool, int64_t, int64_t, int, int, const float *, T *, hipStream_t);         \
    template void launch_spin_mean<T>(const T *, int64_t, int64_t, int, int, int, int, int, T *, hipStream_t);      \
    template void launch_layer_epi<T>(const T *, const T *, const T *, const T *, T *, int64_t, int64_t, int, int,  \
                                      int, int, int, int, bool, T *, hipStream_t);                                  \
    template void launch_envelope<T>(const Sys &, const double *, const T *, int64_t, int64_t, int64_t, int,        \
                                     const T *, int64_t, int64_t, int, bool, double *, hipStream_t);                \
    template void launch_orbdet<T>(const Sys &, const double *, const T *, const OrbSpins<T> &, int64_t, int, bool,  \
                                   double *, int, hipStream_t);                                                     \
    template bool launch_orbdet_combine<T>(const Sys &, const double *, const T *, const OrbSpins<T> &, int64_t,    \
                                           int, double *, int8_t *, const AcceptArgs &, hipStream_t);

FN_INST(float)
FN_INST(double)

}  // namespace fn
