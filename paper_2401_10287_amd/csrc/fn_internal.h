// fn_internal.h -- shared definitions of the gfx950 HIP implementation.
//
// Row layout of every stream activation ("forward-Laplacian rows"): each
// electron of each walker owns TR consecutive rows of a row-major matrix.
//   row 0             value
//   row 1 + c         d/dx_c, c = 3 e + a over all 3N electron coordinates
//   row 3N + 1        Laplacian (sum over all 3N coordinates)
//   rows 3N+2..TR-1   padding (TR is a multiple of 16): zero in the input
//                     features; the fused layer kernel neither fetches nor
//                     writes them, and every consumer either reads rows up
//                     to 3N+1 only or keeps them row-local (a matrix
//                     product's padding output rows are never read into a
//                     live row)
// In value-only mode (Metropolis, gradient) TR = 1.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include "fnvmc.h"

namespace fn {

// System and network sizes, passed to kernels by value.
struct Sys {
    int M, N, nu, nd, L, w1, w2, K;
    int iso;        // isotropic envelope: one sigma per orbital and nucleus (Sigma = sigma I)
    double R[FN_MAX_NUC][3];
    double Z[FN_MAX_NUC];
};

inline __host__ __device__ int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Offsets of the parameter tensors in the flat vector (same layout as the
// header comment of fnvmc.h).
struct ParamLayout {
    int64_t V[FN_MAX_LAYERS], b[FN_MAX_LAYERS], W2[FN_MAX_LAYERS], c2[FN_MAX_LAYERS];
    int64_t w[2], g[2], pi[2], sig[2];
    int64_t total;
};

inline __host__ __device__ int layer_dh(const Sys &s, int l) { return l == 0 ? 4 * s.M : s.w1; }
inline __host__ __device__ int layer_dp(const Sys &s, int l) { return l == 0 ? 4 : s.w2; }
inline __host__ __device__ int layer_din(const Sys &s, int l) { return 3 * layer_dh(s, l) + 2 * layer_dp(s, l); }
// envelope parameter partials per (orbital column, nucleus) in the backward:
// pi and the nine entries of Sigma, or pi and sigma
inline __host__ __device__ int env_partials(const Sys &s) { return s.iso ? 2 : 10; }

inline ParamLayout make_layout(const Sys &s)
{
    ParamLayout p{};
    int64_t o = 0;
    for (int l = 0; l < s.L; ++l) {
        p.V[l] = o; o += (int64_t)layer_din(s, l) * s.w1;
        p.b[l] = o; o += s.w1;
    }
    for (int l = 0; l + 1 < s.L; ++l) {
        p.W2[l] = o; o += (int64_t)layer_dp(s, l) * s.w2;
        p.c2[l] = o; o += s.w2;
    }
    for (int sp = 0; sp < 2; ++sp) {
        int n = sp == 0 ? s.nu : s.nd;
        if (n == 0) { p.w[sp] = p.g[sp] = p.pi[sp] = p.sig[sp] = -1; continue; }
        int kn = s.K * n;
        p.w[sp] = o; o += (int64_t)s.w1 * kn;
        p.g[sp] = o; o += kn;
        p.pi[sp] = o; o += (int64_t)kn * s.M;
        p.sig[sp] = o; o += (int64_t)kn * s.M * (s.iso ? 1 : 9);
    }
    p.total = o;
    return p;
}

// Matrix-product arithmetic.
//   GEMM_BF16W3 / GEMM_BF16W2: BF16 weights (the parameters rounded to
//   nearest even when packed) times FP32 activations split into three (exact)
//   or two BF16 parts: one product per activation part.
enum GemmMode { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16 = 2, GEMM_BF16X3 = 3, GEMM_BF16X6 = 4, GEMM_BF16W3 = 5,
                GEMM_BF16W2 = 6 };

// BF16 parts of the activation operand and of the weight operand of a mode
// (1 for the FP32 / FP64 modes)
__host__ __device__ constexpr int act_parts(int m)
{
    return m == GEMM_BF16X3 || m == GEMM_BF16W2 ? 2 : (m == GEMM_BF16X6 || m == GEMM_BF16W3 ? 3 : 1);
}
__host__ __device__ constexpr int weight_parts(int m) { return m == GEMM_BF16X3 ? 2 : (m == GEMM_BF16X6 ? 3 : 1); }
// modes whose products run on the BF16 matrix instructions
__host__ __device__ constexpr bool split_mode(int m) { return m >= GEMM_BF16 && m <= GEMM_BF16W2; }
// modes whose weights are the BF16 roundings of the parameters
__host__ __device__ constexpr bool bf16_weight_mode(int m) { return m == GEMM_BF16W3 || m == GEMM_BF16W2; }

// f(std::integral_constant<int, MODE>{}) for a split-BF16 mode known at run time
template <typename F>
inline void with_split_mode(int mode, F &&f)
{
    switch (mode) {
    case GEMM_BF16: f(std::integral_constant<int, GEMM_BF16>{}); break;
    case GEMM_BF16X3: f(std::integral_constant<int, GEMM_BF16X3>{}); break;
    case GEMM_BF16W3: f(std::integral_constant<int, GEMM_BF16W3>{}); break;
    case GEMM_BF16W2: f(std::integral_constant<int, GEMM_BF16W2>{}); break;
    default: f(std::integral_constant<int, GEMM_BF16X6>{}); break;
    }
}

// LDS layout of the BF16 operand tiles of the matrix-core kernels: rows of
// 32 elements (four 16-byte chunks, no padding), chunk c of row r stored in
// slot c ^ s(r), s(r) = ((r >> 1) ^ (r >> 2)) & 3.  Row stores in 8- or
// 16-byte pieces and 16-byte fragment reads of 16 consecutive rows at one
// chunk then fall on distinct banks.
__host__ __device__ inline int lds_chunk(int r, int c) { return c ^ (((r >> 1) ^ (r >> 2)) & 3); }

typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;     // one 16 x 16 MFMA accumulator per lane
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;     // one BF16 MFMA operand fragment

// Split two FP32 values a, b into NP BF16 parts, x = p0 + p1 + ..., each part
// the round-to-nearest-even of what the earlier parts leave (NaN stays NaN).
// Part q of both values comes back packed in h[q], a in the low half; one
// packed hardware conversion per part.
template <int NP>
__device__ inline void split_bf16_pair(float a, float b, uint32_t (&h)[NP])
{
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const f32x2_t v = {a, b};
        const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
        h[q] = w;
        if (q + 1 < NP) {
            a -= __uint_as_float(w << 16);
            b -= __uint_as_float(w & 0xffff0000u);
        }
    }
}

// v rounded to the nearest BF16 value, ties to even (NaN stays NaN): the
// weights of the BF16-weight modes
__device__ inline float bf16_round(float v)
{
    const uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return v;
    return __uint_as_float(((u + 0x7fffu + ((u >> 16) & 1u)) >> 16) << 16);
}

// Direct global-to-LDS staging of operand tiles (split-BF16 products).
// copy16_to_lds: each lane copies 16 bytes from its own global address g to
// lds + 16 * lane (lds: the wave's 1 KB block, the same for all lanes).
// wait_copies: until this lane's copies have landed (vmcnt(0) with the other
// counters left alone; a barrier after it makes every lane's copies visible).
__device__ inline void copy16_to_lds(const void *g, void *lds)
{
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}
__device__ inline void wait_copies() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The NP BF16 parts of one MFMA A fragment: eight consecutive FP32 values
// (x0 then x1) of one row, split with split_bf16_pair.
template <int NP>
__device__ inline void split_fragment(float4 x0, float4 x1, bf16x8 (&h)[NP])
{
    uint32_t p0[NP], p1[NP], p2[NP], p3[NP];
    split_bf16_pair<NP>(x0.x, x0.y, p0);
    split_bf16_pair<NP>(x0.z, x0.w, p1);
    split_bf16_pair<NP>(x1.x, x1.y, p2);
    split_bf16_pair<NP>(x1.z, x1.w, p3);
#pragma unroll
    for (int q = 0; q < NP; ++q) h[q] = __builtin_bit_cast(bf16x8, make_uint4(p0[q], p1[q], p2[q], p3[q]));
}

// Products of one reduction step, activation fragments in NA BF16 parts and
// weight fragments in NW parts, for the first NI of WI row blocks.  Equal
// splits: the pairs (pa, pb) with pa + pb < NA, the smallest terms first
// (pa + pb descending).  One weight part (BF16 weights): pa = 0 .. NA - 1, so
// the first group needs only the leading activation part.
template <int NA, int NW, int NI, int WI, int WJ>
__device__ __forceinline__ void split_products(const bf16x8 (&ha)[NA][WI], const bf16x8 (&hb)[NW][WJ],
                                               f32x4 (&acc)[WI][WJ])
{
    static_assert(NW == NA || NW == 1, "split pairing");
    if constexpr (NW == 1) {
#pragma unroll
        for (int pa = 0; pa < NA; ++pa)
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < WJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[pa][i], hb[0][j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
        for (int sum = NA - 1; sum >= 0; --sum)
#pragma unroll
            for (int pa = 0; pa <= sum; ++pa)
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = 0; j < WJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[pa][i], hb[sum - pa][j], acc[i][j],
                                                                            0, 0, 0);
    }
}
__host__ __device__ constexpr int split_product_count(int na, int nw) { return nw == 1 ? na : na * (na + 1) / 2; }

// Scheduling hint for a reduction step of NB x NJ accumulator blocks with
// activations in NA parts and weights in NW parts: the first part's
// conversions (4 per row block), then each matrix instruction of the first
// NA - 1 product groups followed by a share of the next parts' conversions
// (about 20 vector instructions per row block and part), then the remaining
// matrix instructions.
constexpr int SCHED_VALU = 0x002, SCHED_MFMA = 0x008;
template <int NA, int NW, int NB, int NJ>
__device__ inline void sched_split_products()
{
    constexpr int G = NB * NJ, VM = (20 * NB + G - 1) / G;
    __builtin_amdgcn_sched_group_barrier(SCHED_VALU, 4 * NB, 0);
#pragma unroll
    for (int g = 0; g < NA - 1; ++g)
#pragma unroll
        for (int m = 0; m < G; ++m) {
            __builtin_amdgcn_sched_group_barrier(SCHED_MFMA, 1, 0);
            __builtin_amdgcn_sched_group_barrier(SCHED_VALU, VM, 0);
        }
    __builtin_amdgcn_sched_group_barrier(SCHED_MFMA, G * (split_product_count(NA, NW) - (NA - 1)), 0);
}

// bitwise select (m all ones or zero) of a float4
__device__ inline float4 mask4f(float4 x, uint32_t m)
{
    return make_float4(__uint_as_float(__float_as_uint(x.x) & m), __uint_as_float(__float_as_uint(x.y) & m),
                       __uint_as_float(__float_as_uint(x.z) & m), __uint_as_float(__float_as_uint(x.w) & m));
}

// Split-reduction tile of the small-grid products (activations in NA and
// weights in NW BF16 parts): the
// 32 x 32 output tile at (m0, n0) of [A1 | A2] W^T, the 32-wide reduction
// steps split over the workgroup's four waves in contiguous quarters.  Each
// wave loads its operand fragments straight from global memory into
// registers (the next step's loads issued before the current step's matrix
// instructions) and multiplies the parts in the order of the tiled kernels;
// acc is this wave's partial tile, accumulator (i, j) element e at row
// 16 i + 4 (lane / 16) + e, column 16 j + lane % 16.  arow(r): A's row of
// product row r.  Rows past `rows` and columns past nout load row m0 /
// column n0 and are zeroed.  A1 / A2 FP32 row-major; W NW parts of BF16
// rows of ldw (part stride wpart); K1, K2 multiples of 32.
template <int NA, int NW, typename ARow>
__device__ __forceinline__ void splitk_accumulate(const float *A1, int64_t lda1, int K1, const float *A2, int64_t lda2,
                                                  int K2, const uint16_t *W, int64_t wpart, int64_t ldw, int nout,
                                                  int64_t rows, int64_t m0, int n0, ARow arow, f32x4 (&acc)[2][2])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ksteps = (K1 + K2) / 32;
    const int per = (ksteps + 3) / 4;
    const int k0 = wave * per, k1 = min(ksteps, k0 + per);
    const int li = lane & 15, kq = lane >> 4;          // row / column li of a block, reduction offset 8 kq
    int64_t ar[2], wr[2];
    uint32_t am[2], wm[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t r = m0 + 16 * i + li;
        am[i] = r < rows ? 0xffffffffu : 0u;
        ar[i] = arow(r < rows ? r : m0);
        const int o = n0 + 16 * i + li;
        wm[i] = o < nout ? 0xffffffffu : 0u;
        wr[i] = (int64_t)(o < nout ? o : n0) * ldw;
    }
    float4 xa[2][2], na[2][2];
    uint4 xb[2][NW], nb[2][NW];
    auto load = [&](int kt, float4 (&A)[2][2], uint4 (&Bv)[2][NW]) {
        const int kb = kt * 32;
        const bool first = kb < K1;
        const float *base = first ? A1 : A2;
        const int64_t lda = first ? lda1 : lda2;
        const int kk = (first ? kb : kb - K1) + 8 * kq;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float *pa = base + ar[i] * lda + kk;
            A[i][0] = *(const float4 *)pa;
            A[i][1] = *(const float4 *)(pa + 4);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < NW; ++q) Bv[j][q] = *(const uint4 *)(W + (int64_t)q * wpart + wr[j] + kb + 8 * kq);
    };
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (k0 < k1) load(k0, xa, xb);
    for (int kt = k0; kt < k1; ++kt) {
        if (kt + 1 < k1) load(kt + 1, na, nb);
        bf16x8 ha[NA][2], hb[NW][2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x8 hp[NA];
            split_fragment<NA>(mask4f(xa[i][0], am[i]), mask4f(xa[i][1], am[i]), hp);
#pragma unroll
            for (int q = 0; q < NA; ++q) ha[q][i] = hp[q];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint4 u = xb[j][q];
                hb[q][j] = __builtin_bit_cast(bf16x8, make_uint4(u.x & wm[j], u.y & wm[j], u.z & wm[j], u.w & wm[j]));
            }
        split_products<NA, NW, 2, 2, 2>(ha, hb, acc);
        if (kt + 1 < k1) {
#pragma unroll
            for (int i = 0; i < 2; ++i) { xa[i][0] = na[i][0]; xa[i][1] = na[i][1]; }
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < NW; ++q) xb[j][q] = nb[j][q];
        }
    }
}

// each wave's partial tile into red[wave]; returns after a workgroup barrier
__device__ __forceinline__ void splitk_park(const f32x4 (&acc)[2][2], float (&red)[4][32][33])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[wave][16 * i + 4 * kq + e][16 * j + li] = acc[i][j][e];
    __syncthreads();
}


// Padded widths.  Every product's reduction dimension is a multiple of 32.
struct Widths {
    int HWl[FN_MAX_LAYERS];   // padded width of the h_i block of layer l
    int GWl[FN_MAX_LAYERS];   // padded width of [g_i_up | g_i_dn] of layer l
    int HWmax, GWmax, W1p;    // buffer strides
    int KNp[2];               // K n_s padded to 32 (head outputs)
};

inline Widths make_widths(const Sys &s)
{
    Widths w{};
    w.HWmax = 0;
    w.GWmax = 0;
    for (int l = 0; l < s.L; ++l) {
        w.HWl[l] = round_up(layer_dh(s, l), 32);
        w.GWl[l] = round_up(2 * layer_dp(s, l), 32);
        if (w.HWl[l] > w.HWmax) w.HWmax = w.HWl[l];
        if (w.GWl[l] > w.GWmax) w.GWmax = w.GWl[l];
    }
    w.W1p = round_up(s.w1, 32);
    if (w.W1p > w.HWmax) w.HWmax = w.W1p;
    for (int sp = 0; sp < 2; ++sp) w.KNp[sp] = round_up(s.K * (sp == 0 ? s.nu : s.nd), 32);
    return w;
}

// Arguments of one matrix product C[r][o] = sum_k A[r][k] W[o][k] where A is
// the row-wise concatenation [A1 | A2] (A2 may be empty) and W is stored
// transposed (o major, k contiguous) in the product's operand type.  Row r of
// A: group g = r / rows_per_group, q = r % rows_per_group, A's row is
// g * group_stride + row_offset + q, where, when rows_per_inner > 0, q itself
// is mapped to (q / rows_per_inner) * inner_stride + q % rows_per_inner (the
// live rows of each electron of one spin, say).  C's row is r, or, when
// c_rows_per_group > 0, the one-level mapping with the c_ fields.
struct GemmArgs {
    const void *A1; int64_t lda1; int K1;
    const void *A2; int64_t lda2; int K2;
    const void *W; int64_t wpart; int64_t ldw;   // BF16 modes: parts at W + q * wpart
    void *C; int64_t ldc;
    int64_t rows; int nout;
    int64_t rows_per_group, group_stride, row_offset;
    int64_t c_rows_per_group, c_group_stride, c_row_offset;
    int64_t rows_per_inner, inner_stride;
};

// A's row for product row r (see GemmArgs)
__host__ __device__ inline int64_t gemm_a_row(const GemmArgs &a, int64_t r)
{
    const int64_t g = r / a.rows_per_group;
    int64_t q = r - g * a.rows_per_group;
    if (a.rows_per_inner > 0) {
        const int64_t e = q / a.rows_per_inner;
        q = e * a.inner_stride + (q - e * a.rows_per_inner);
    }
    return g * a.group_stride + a.row_offset + q;
}

// Block order for a grid of row blocks x ncb column blocks (ncb = 1 or 2):
// workgroups are dealt to the eight XCDs in turn, so the two column halves of
// one row block get ids that differ by 8 -- same XCD, adjacent in time -- and
// the second half finds the rows in that XCD's L2.
__host__ __device__ inline void xcd_tile(int64_t b, int ncb, int64_t &rb, int &cb)
{
    if (ncb == 1) { rb = b; cb = 0; return; }
    const int64_t hi = b >> 4, rem = b & 15;
    cb = (int)(rem >> 3);
    rb = hi * 8 + (rem & 7);
}

inline int64_t xcd_grid(int64_t nrb, int ncb) { return ncb == 1 ? nrb : ((nrb + 7) / 8) * 16; }

__host__ __device__ inline int64_t remap_row(int64_t r, int64_t per, int64_t stride, int64_t off)
{
    // 32-bit division when both fit (the common case; 64-bit division is a long sequence on the GPU)
    const int64_t g = ((r | per) >> 31) == 0 ? (int64_t)((uint32_t)r / (uint32_t)per) : r / per;
    return g * stride + off + (r - g * per);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter c -> c, key
// (k0, k1); the sampler's generator
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// 53 random bits from two words, mapped to (0, 1]
__device__ inline double word_pair_to_unit(uint32_t a, uint32_t b)
{
    const uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(m + 1) * 0x1.0p-53;
}

// records msg as the calling thread's fn_last_error() message; returns st
fn_status api_fail(fn_status st, const char *msg);

hipError_t launch_gemm(int mode, const GemmArgs &a, hipStream_t st);
// two products in one launch when they take the same tile shape (else two
// launches); each product's results are those of launch_gemm
hipError_t launch_gemm2(int mode, const GemmArgs &a0, const GemmArgs &a1, hipStream_t st);

// One fused one-electron stream layer (product + forward-Laplacian tanh
// epilogue + residual).  A1 = h^l (rows of TR per electron, also the residual
// source), A2 = pair means of layer l, W = packed V_h (nout = w1 columns),
// Pw = per-walker part [walker * TR + t][w1], bias = b_l.
struct LayerArgs {
    const float *A1; int64_t lda1; int K1;
    const float *A2; int64_t lda2; int K2;
    const void *W; int64_t wpart; int64_t ldw; int nout;
    const float *Pw; const float *bias;
    float *Hout; int64_t ldh_out;
    int64_t rows; int N; int n3; int w1; int W1p; int resid;
    // when a 128-row tile holds whole walkers (N * TR divides 128): also
    // write the next layer's spin means [g_up | g_dn] of h^{l+1}, rows
    // walker * TR + t for t up to the Laplacian row (padding rows are not
    // written), ld 2 * W1p (Gout = nullptr: skip)
    float *Gout; int nu;
};

bool stream_layer_supported(int mode, int TR, int w1, int W1p);
extern bool g_use_fused_layer;
extern bool g_layer_dma;
extern bool g_gemm_wide;     // 96-column product tiles (tuning switch "gemm_wide")
extern bool g_gemm_splitk;   // split-K kernel for small-grid products (tuning switch "gemm_splitk")
// set for the duration of a grouped call on the calling thread: the
// split-reduction kernels are not chosen, so a walker's arithmetic does not
// depend on the batch size
extern thread_local bool g_splitk_suppressed;
// pair-stream launch shape: output columns per thread (0: by size) and
// (pair, column group) items per workgroup (0: by form)
extern int g_pair_oc, g_pair_items;
extern int g_det_stage;     // determinant kernels: envelope parameters staged in LDS where they fit
// FP32 pair layers on the matrix cores (false: vector kernel)
extern bool g_pair_mfma;
void launch_stream_layer(int mode, const LayerArgs &a, int TR, hipStream_t st);

// Every one-electron layer of a forward-Laplacian pass in one kernel
// (fn_stack.hip), for two to four electrons (TR = 16) and w1 = 256.
struct StackArgs {
    const float *H0; int64_t ldh;             // features of layer 0 (rows walker * N * 16 + e * 16 + t)
    const float *GI; int64_t ldgi; int64_t gi_stride;   // pair means of every layer (layer stride in floats)
    const uint16_t *Wx[FN_MAX_LAYERS], *Wg[FN_MAX_LAYERS];   // packed split-BF16 V_h / V_g per layer
    const float *Wx32[FN_MAX_LAYERS], *Wg32[FN_MAX_LAYERS];  // the same transposed, FP32 (six-product split)
    int64_t wxpart[FN_MAX_LAYERS], wgpart[FN_MAX_LAYERS];
    int HW[FN_MAX_LAYERS], GW[FN_MAX_LAYERS];  // padded widths of h and of [g_i_up | g_i_dn]
    const float *bias[FN_MAX_LAYERS];
    float *Hout;                               // h^L, live rows, leading dimension ldh
    int64_t B; int L; int nu; int n3;
    // the orbital head in the register kernel (WH[0] non-null): BF16 head
    // weights per spin, [32 = K n][ldwh], and the outputs O[spin] (rows
    // (walker n + j) 16 + t, leading dimension ldo[spin]); Hout unused then
    const uint16_t *WH[2]; int ldwh; float *O[2]; int64_t ldo[2];
};
extern int g_use_stack;                        // tuning switch "layer_stack": 0 never, 1 one-pass BF16, 2 every split mode
extern int g_stack_shape;                      // tuning switch "stack_shape": workgroup shape 0, 1, 2
bool stack_supported(int mode, int N, int TR, int w1, int L);
// the stacked kernel of the six-product split reads FP32 weights and splits
// them in registers (one copy of every layer's weights fits in L2)
inline bool stack_fp32_weights(int mode) { return mode == GEMM_BF16X6; }
void launch_stack(int mode, const StackArgs &a, int N, hipStream_t st);
// Every one-electron layer with the activations in registers (fn_stackr.hip):
// four electrons, two per spin, w1 = 256, modes with one BF16 weight part
// (tuning switch "stack_regs", on by default)
extern bool g_stack_regs;
bool stack_regs_supported(int mode, int N, int nu, int TR, int w1, int L, const int *HW, const int *GW);
// the orbital head fused into it: one BF16 weight part, K n = 32 per spin, w1 = 256
inline bool stack_regs_head(int mode, int hmode, int K, int nu, int nd, int W1p)
{
    return hmode == mode && (mode == GEMM_BF16W3 || mode == GEMM_BF16W2) && K * nu == 32 && K * nd == 32 && W1p == 256;
}
void launch_stack_regs(int mode, const StackArgs &a, hipStream_t st);
// 128-row tiles of the fused layer hold whole walkers
inline bool stream_layer_whole_walkers(int N, int TR) { return N * TR <= 128 && 128 % (N * TR) == 0; }

// Rows per electron in forward-Laplacian form: 3N + 2 rounded up to the next
// power of two up to 64 (N <= 20), the row counts whose electrons tile the
// fused layer kernel's 128-row blocks; beyond that, rounded up to 16.
inline int fl_rows(int N)
{
    const int t = 3 * N + 2;
    int p2 = 16;
    while (p2 < t) p2 *= 2;
    return p2 <= 64 ? p2 : round_up(t, 16);
}

}  // namespace fn
