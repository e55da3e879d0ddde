// fn_gemm.hip -- matrix products of the stream layers and the orbital head.
//
// C[r][o] = sum_k [A1 | A2][r][k] W[o][k]: the dense contraction of every
// one-electron layer (its per-electron part and its per-walker mean-field
// part) and of the orbital head, over forward-Laplacian rows (value, 3N
// tangents, Laplacian) of all walkers at once.
//
// gfx950 matrix cores: one 256-thread workgroup owns a 128 x 128 output tile;
// each of its four wave64s owns a 64 x 64 quarter as 4 x 4 blocks of 16 x 16
// accumulators.  Operand tiles of 32 reduction steps are staged through LDS
// (the A tile converted from FP32 to the product's operand type on the way in)
// and the next tile's global loads are issued before the current tile's
// matrix instructions.  128-column tiles in the split-BF16 modes copy their
// operand tiles straight from global memory into a two-stage LDS ring
// instead, and each wave splits its activation fragments as it reads them.
//   GEMM_F32    v_mfma_f32_16x16x4_f32, FP32 operands
//   GEMM_BF16   v_mfma_f32_16x16x32_bf16, BF16 operands (round to nearest even)
//   GEMM_BF16X3 x = hi + lo split of each FP32 operand, hi*hi + hi*lo + lo*hi
//   GEMM_BF16X6 x = hi + mid + lo split, the six products whose part indices
//               sum to at most 2 (FP32-level operand precision)
//   GEMM_BF16W3 BF16 weights (the parameters rounded to nearest even) times
//               the exact hi + mid + lo split of the FP32 activations: three
//               products, each exact, accumulated in FP32
//   GEMM_BF16W2 BF16 weights times the hi + lo split of the activations
//   GEMM_F64    FP64 on the vector ALUs (64 x 64 tiles)
#include "fn_internal.h"

namespace fn {

bool g_gemm_splitk = true;
thread_local bool g_splitk_suppressed = false;
// 96-column tiles for outputs of 65..96 columns (tuning switch "gemm_wide";
// otherwise 128-column tiles); each output element takes the same
// arithmetic whatever the tile width.  (160-column tiles for 129..160, one
// workgroup per CU in the split-BF16 modes, measured slower than two
// 128-column tiles.)
bool g_gemm_wide = true;


constexpr int BM = 128, BK = 32;

constexpr int LDH = BK;       // LDS row stride of BF16 tiles (64 bytes, chunk-swizzled by lds_chunk)
constexpr int LDF = BK + 4;   // LDS row stride of FP32 tiles (144 bytes)

template <int MODE>
struct ModeInfo {
    static constexpr bool F32 = MODE == GEMM_F32;
    static constexpr int NA = act_parts(MODE);      // BF16 parts of the activation operand
    static constexpr int NW = weight_parts(MODE);   // BF16 parts of the weight operand
};

// DMA (split-BF16 modes, 128-column tiles, K1 a multiple of 32): operand
// tiles by direct global-to-LDS copies into a two-stage ring, FP32
// activations split by each wave as it reads its fragments (the layout of
// the fused layer kernel's staged path); bitwise equal to the register path.
template <int MODE, int BNT, bool DMA>
__device__ __forceinline__ void gemm_tile(const GemmArgs &a, int64_t bid)
{
    constexpr bool F32 = ModeInfo<MODE>::F32;
    constexpr int NA = ModeInfo<MODE>::NA, NW = ModeInfo<MODE>::NW;
    static_assert(!DMA || (BNT == 128 && !F32), "staged copies");
    // wave tiling: 2 x 2 waves of 64 x 64 for 128 columns, else 4 x 1 waves of 32 x BNT
    constexpr int WI = BNT == 128 ? 4 : 2;          // 16-row blocks per wave
    constexpr int WJ = BNT == 128 ? 4 : BNT / 16;   // 16-column blocks per wave
    constexpr int AST = BM * BK * 4, STG = AST + NW * BNT * BK * 2;
    __shared__ __attribute__((aligned(16))) float sAf[F32 ? BM * LDF : 1];
    __shared__ __attribute__((aligned(16))) float sBf[F32 ? BNT * LDF : 1];
    __shared__ __attribute__((aligned(16))) uint16_t sAh[F32 || DMA ? 8 : NA * BM * LDH];
    __shared__ __attribute__((aligned(16))) uint16_t sBh[F32 || DMA ? 8 : NW * BNT * LDH];
    __shared__ __attribute__((aligned(16))) unsigned char sR[DMA ? 2 * STG : 16];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = BNT == 128 ? wave >> 1 : wave, wn = BNT == 128 ? wave & 1 : 0;
    const int ncb = (a.nout + BNT - 1) / BNT;
    int64_t rb;
    int cb;
    if (ncb <= 2) {
        xcd_tile(bid, ncb, rb, cb);
    } else {
        rb = bid % ((a.rows + BM - 1) / BM);
        cb = (int)(bid / ((a.rows + BM - 1) / BM));
    }
    const int64_t m0 = rb * BM;
    const int n0 = cb * BNT;
    if (m0 >= a.rows || n0 >= a.nout) return;
    const int ktiles = (a.K1 + a.K2) / BK;

    // A rows loaded by this thread: 4 float4 per tile, row = f >> 3, k4 = f & 7
    int64_t arow[4];
    bool aval[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        int f = tid + 256 * v;
        int64_t r = m0 + (f >> 3);
        aval[v] = r < a.rows;
        arow[v] = gemm_a_row(a, r);
    }
    const float *A1 = (const float *)a.A1;
    const float *A2 = (const float *)a.A2;

    constexpr int NWF = F32 ? (BNT * 8 + 255) / 256 : 1;      // float4 of B per thread
    constexpr int NWH = F32 ? 1 : (BNT * 4 + 255) / 256;      // uint4 of B per thread per part
    float4 ra[4];
    uint4 rwh[F32 ? 1 : NWH * NW];
    float4 rwf[NWF];

    auto load_tile = [&](int kt) {
        const int kb = kt * BK;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int f = tid + 256 * v;
            int k = kb + 4 * (f & 7);
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (aval[v]) {
                const float *p = k < a.K1 ? A1 + arow[v] * a.lda1 + k : A2 + arow[v] * a.lda2 + (k - a.K1);
                val = *(const float4 *)p;
            }
            ra[v] = val;
        }
        if constexpr (F32) {
            const float *W = (const float *)a.W;
#pragma unroll
            for (int v = 0; v < NWF; ++v) {
                int f = tid + 256 * v;
                int o = n0 + (f >> 3);
                rwf[v] = (f < BNT * 8 && o < a.nout) ? *(const float4 *)(W + (int64_t)o * a.ldw + kb + 4 * (f & 7))
                                                     : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
            // the NW weight parts are stored one after another, part stride a.wpart elements
            const uint16_t *W = (const uint16_t *)a.W;
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int v = 0; v < NWH; ++v) {
                    int f = tid + 256 * v;
                    int o = n0 + (f >> 2);
                    int64_t off = (int64_t)q * a.wpart + (int64_t)o * a.ldw + kb + 8 * (f & 3);
                    rwh[q * NWH + v] = (f < BNT * 4 && o < a.nout) ? *(const uint4 *)(W + off) : make_uint4(0, 0, 0, 0);
                }
        }
    };

    auto store_tile = [&]() {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int f = tid + 256 * v;
            int r = f >> 3, k = 4 * (f & 7);
            float4 x = ra[v];
            if constexpr (F32) {
                *(float4 *)&sAf[r * LDF + k] = x;
            } else {
                uint32_t h01[NA], h23[NA];
                split_bf16_pair<NA>(x.x, x.y, h01);
                split_bf16_pair<NA>(x.z, x.w, h23);
#pragma unroll
                for (int q = 0; q < NA; ++q)
                    *(uint2 *)&sAh[q * BM * LDH + r * LDH + 8 * lds_chunk(r, k >> 3) + (k & 7)] = make_uint2(h01[q], h23[q]);
            }
        }
        if constexpr (F32) {
#pragma unroll
            for (int v = 0; v < NWF; ++v) {
                int f = tid + 256 * v;
                if (f < BNT * 8) *(float4 *)&sBf[(f >> 3) * LDF + 4 * (f & 7)] = rwf[v];
            }
        } else {
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int v = 0; v < NWH; ++v) {
                    int f = tid + 256 * v;
                    if (f < BNT * 4) *(uint4 *)&sBh[q * BNT * LDH + (f >> 2) * LDH + 8 * lds_chunk(f >> 2, f & 3)] = rwh[q * NWH + v];
                }
        }
    };

    f32x4 acc[WI][WJ];
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (DMA) {
        // per lane: its 16-byte chunk of each of the wave's 1 KB blocks
        // (activations: 4 blocks of 8 rows, chunk c of row r at c ^ (r & 7);
        // weights: 2 blocks of 16 rows per part, chunk c at lds_chunk(r, c)).
        // Rows past the end copy row m0 and weight rows past nout copy row
        // n0; they only feed outputs that are not stored.
        int64_t da1[4], da2[4], dw[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 8 * (4 * wave + j) + (lane >> 3);
            const int c = (lane & 7) ^ (r & 7);
            const int64_t rr = m0 + r < a.rows ? m0 + r : m0;
            const int64_t ar = gemm_a_row(a, rr);
            da1[j] = ar * a.lda1 + 4 * c;
            da2[j] = ar * a.lda2 + 4 * c;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int r = 16 * (2 * wave + j) + (lane >> 2);
            const int o = n0 + r;
            dw[j] = (int64_t)(o < a.nout ? o : n0) * a.ldw + 8 * lds_chunk(r, lane & 3);
        }
        auto dma = [&](int kt, int sgi) {
            const int kb = kt * BK;
            unsigned char *stg = sR + sgi * STG;
            const float *base = kb < a.K1 ? A1 + kb : A2 + (kb - a.K1);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                copy16_to_lds(base + (kb < a.K1 ? da1[j] : da2[j]), stg + (4 * wave + j) * 1024);
            const uint16_t *W = (const uint16_t *)a.W + kb;
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    copy16_to_lds(W + (int64_t)q * a.wpart + dw[j], stg + AST + q * BNT * BK * 2 + (2 * wave + j) * 1024);
        };
        if (ktiles > 0) dma(0, 0);
        const int ar = wm * 16 * WI + (lane & 15), br = wn * 16 * WJ + (lane & 15);
        const int ko = 8 * lds_chunk(lane & 15, lane >> 4);
        const int h = lane >> 4, sw = lane & 7;
        for (int kt = 0; kt < ktiles; ++kt) {
            wait_copies();                           // this lane's copies of step kt have landed
            __syncthreads();                         // everyone's have; step kt - 1's stage is free
            const unsigned char *stg = sR + (kt & 1) * STG;
            const float *sA = (const float *)stg;
            const uint16_t *sB = (const uint16_t *)(stg + AST);
            float4 xa[WI][2];
            bf16x8 ha[NA][WI], hb[NW][WJ];
#pragma unroll
            for (int i = 0; i < WI; ++i) {
                const float *rowp = sA + (ar + 16 * i) * BK;
                xa[i][0] = *(const float4 *)(rowp + 4 * ((2 * h) ^ sw));
                xa[i][1] = *(const float4 *)(rowp + 4 * ((2 * h + 1) ^ sw));
            }
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int j = 0; j < WJ; ++j) hb[q][j] = *(const bf16x8 *)&sB[q * BNT * LDH + (br + 16 * j) * LDH + ko];
            if (kt + 1 < ktiles) dma(kt + 1, (kt + 1) & 1);
            // split and multiply at raised wave priority: this wave's matrix
            // instructions issue ahead of the other workgroup's on the SIMD,
            // whose fragment reads and copies then fill the gaps
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < WI; ++i) {
                bf16x8 hp[NA];
                split_fragment<NA>(xa[i][0], xa[i][1], hp);
#pragma unroll
                for (int q = 0; q < NA; ++q) ha[q][i] = hp[q];
            }
            split_products<NA, NW, WI, WI, WJ>(ha, hb, acc);
            sched_split_products<NA, NW, WI, WJ>();
            __builtin_amdgcn_s_setprio(0);
        }
    } else {
    if (ktiles > 0) load_tile(0);
    for (int kt = 0; kt < ktiles; ++kt) {
        __syncthreads();
        store_tile();
        __syncthreads();
        if (kt + 1 < ktiles) load_tile(kt + 1);
        const int ar = wm * 16 * WI + (lane & 15), br = wn * 16 * WJ + (lane & 15);
        if constexpr (F32) {
#pragma unroll
            for (int kk = 0; kk < BK / 4; ++kk) {
                float fa[WI], fb[WJ];
#pragma unroll
                for (int i = 0; i < WI; ++i) fa[i] = sAf[(ar + 16 * i) * LDF + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int j = 0; j < WJ; ++j) fb[j] = sBf[(br + 16 * j) * LDF + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int i = 0; i < WI; ++i)
#pragma unroll
                    for (int j = 0; j < WJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        } else {
            const int ko = 8 * lds_chunk(lane & 15, lane >> 4);   // rows ar + 16 i, br + 16 j share bits 0-3 with lane
            bf16x8 ha[NA][WI], hb[NW][WJ];
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int i = 0; i < WI; ++i) ha[q][i] = *(const bf16x8 *)&sAh[q * BM * LDH + (ar + 16 * i) * LDH + ko];
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int j = 0; j < WJ; ++j) hb[q][j] = *(const bf16x8 *)&sBh[q * BNT * LDH + (br + 16 * j) * LDH + ko];
            split_products<NA, NW, WI, WI, WJ>(ha, hb, acc);
        }
    }
    }

    // accumulator (i, j) element e sits at row 16 i + 4 (lane >> 4) + e, column 16 j + (lane & 15)
    // (each output row is mapped once)
    float *C = (float *)a.C;
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int64_t row = m0 + wm * 16 * WI + 16 * i + 4 * (lane >> 4) + e;
            if (row >= a.rows) continue;
            if (a.c_rows_per_group > 0) row = remap_row(row, a.c_rows_per_group, a.c_group_stride, a.c_row_offset);
            float *crow = C + row * a.ldc;
#pragma unroll
            for (int j = 0; j < WJ; ++j) {
                const int col = n0 + wn * 16 * WJ + 16 * j + (lane & 15);
                if (col < a.nout) crow[col] = acc[i][j][e];
            }
        }
}

template <int MODE, int BNT, bool DMA>
__global__ __launch_bounds__(256) void k_gemm_mfma(GemmArgs a)
{
    gemm_tile<MODE, BNT, DMA>(a, blockIdx.x);
}

// two products of one tile shape in one launch: workgroups [0, nb0) take a0,
// the rest a1 (the two spins of the orbital head)
template <int MODE, int BNT, bool DMA>
__global__ __launch_bounds__(256) void k_gemm_mfma2(GemmArgs a0, GemmArgs a1, int64_t nb0)
{
    if ((int64_t)blockIdx.x < nb0) gemm_tile<MODE, BNT, DMA>(a0, blockIdx.x);
    else gemm_tile<MODE, BNT, DMA>(a1, (int64_t)blockIdx.x - nb0);
}

// Small products (split-BF16 modes, grids that would leave most CUs idle):
// one 32 x 32 output tile per 256-thread workgroup with the reduction
// dimension split over its four waves.  Each wave takes a contiguous quarter
// of the 32-wide reduction steps with its operand fragments loaded straight
// from global memory into registers (the next step's loads issued before the
// current step's matrix instructions; products of parts in the order of the
// tiled kernel), and the four partial tiles are summed through LDS in wave
// order.  The chain of dependent reduction steps is a quarter as long.
template <int MODE>
__device__ __forceinline__ void gemm_splitk_tile(const GemmArgs &a, int64_t bid)
{
    constexpr int NA = ModeInfo<MODE>::NA, NW = ModeInfo<MODE>::NW;
    static_assert(MODE != GEMM_F32, "split-BF16 modes");
    __shared__ float red[4][32][33];
    const int tid = threadIdx.x;
    const int64_t nrb = (a.rows + 31) / 32;
    const int64_t m0 = (bid % nrb) * 32;
    const int n0 = (int)(bid / nrb) * 32;
    f32x4 acc[2][2];
    splitk_accumulate<NA, NW>((const float *)a.A1, a.lda1, a.K1, (const float *)a.A2, a.lda2, a.K2,
                          (const uint16_t *)a.W, a.wpart, a.ldw, a.nout, a.rows, m0, n0,
                          [&](int64_t r) { return gemm_a_row(a, r); }, acc);
    splitk_park(acc, red);
    float *C = (float *)a.C;
    for (int q = tid; q < 32 * 32; q += 256) {
        const int r = q >> 5, cc = q & 31;
        int64_t row = m0 + r;
        const int col = n0 + cc;
        if (row >= a.rows || col >= a.nout) continue;
        const float v = ((red[0][r][cc] + red[1][r][cc]) + red[2][r][cc]) + red[3][r][cc];
        if (a.c_rows_per_group > 0) row = remap_row(row, a.c_rows_per_group, a.c_group_stride, a.c_row_offset);
        C[row * a.ldc + col] = v;
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_splitk(GemmArgs a)
{
    gemm_splitk_tile<MODE>(a, blockIdx.x);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_splitk2(GemmArgs a0, GemmArgs a1, int64_t nb0)
{
    if ((int64_t)blockIdx.x < nb0) gemm_splitk_tile<MODE>(a0, blockIdx.x);
    else gemm_splitk_tile<MODE>(a1, (int64_t)blockIdx.x - nb0);
}

// FP64 on the vector ALUs: 64 x 64 tiles, 16-step reduction tiles, 4 x 4
// outputs per thread.
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs a)
{
    __shared__ double sA[16][64 + 1];
    __shared__ double sB[16][64 + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    const int n0 = blockIdx.y * 64;
    const double *A1 = (const double *)a.A1, *A2 = (const double *)a.A2, *W = (const double *)a.W;
    int64_t arow[4];
    bool aval[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        int f = tid + 256 * v;
        int64_t r = m0 + (f >> 4);
        aval[v] = r < a.rows;
        arow[v] = gemm_a_row(a, r);
    }
    double acc[4][4] = {};
    const int K = a.K1 + a.K2;
    for (int kb = 0; kb < K; kb += 16) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int f = tid + 256 * v;
            int r = f >> 4, kk = f & 15, k = kb + kk;
            double x = 0.0;
            if (aval[v]) x = k < a.K1 ? A1[arow[v] * a.lda1 + k] : A2[arow[v] * a.lda2 + (k - a.K1)];
            sA[kk][r] = x;
            int o = n0 + r;
            sB[kk][r] = o < a.nout ? W[(int64_t)o * a.ldw + k] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
    double *C = (double *)a.C;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int64_t row = m0 + ty * 4 + i;
        if (row >= a.rows) continue;
        if (a.c_rows_per_group > 0) row = remap_row(row, a.c_rows_per_group, a.c_group_stride, a.c_row_offset);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int col = n0 + tx * 4 + j;
            if (col < a.nout) C[row * a.ldc + col] = acc[i][j];
        }
    }
}

template <int BNT>
static int64_t bn_grid(const GemmArgs &a)
{
    const int64_t nrb = (a.rows + BM - 1) / BM;
    const int ncb = (a.nout + BNT - 1) / BNT;
    return ncb <= 2 ? xcd_grid(nrb, ncb) : nrb * ncb;
}

template <int MODE, int BNT, bool DMA>
static void launch_kernel(const GemmArgs &a, const GemmArgs *a1, hipStream_t st)
{
    const int64_t g0 = bn_grid<BNT>(a);
    if (a1) {
        const dim3 grid((unsigned)(g0 + bn_grid<BNT>(*a1)));
        hipLaunchKernelGGL((k_gemm_mfma2<MODE, BNT, DMA>), grid, dim3(256), 0, st, a, *a1, g0);
    } else {
        hipLaunchKernelGGL((k_gemm_mfma<MODE, BNT, DMA>), dim3((unsigned)g0), dim3(256), 0, st, a);
    }
}

// a1: a second product of the same tile shape in the same launch, or nullptr
template <int BNT>
static void launch_bn(int mode, const GemmArgs &a, const GemmArgs *a1, hipStream_t st)
{
    if constexpr (BNT == 128) {
        if (g_layer_dma && mode != GEMM_F32 && a.K1 % BK == 0 && (!a1 || a1->K1 % BK == 0)) {
            with_split_mode(mode, [&](auto m) { launch_kernel<decltype(m)::value, 128, true>(a, a1, st); });
            return;
        }
    }
    if (mode == GEMM_F32) launch_kernel<GEMM_F32, BNT, false>(a, a1, st);
    else with_split_mode(mode, [&](auto m) { launch_kernel<decltype(m)::value, BNT, false>(a, a1, st); });
}

// narrowest column tile that covers the output, and narrower still when
// 128-column tiles would leave CUs idle (latency-bound small grids)
static int pick_bn(const GemmArgs &a)
{
    const int64_t nrb = (a.rows + BM - 1) / BM;
    int bn = a.nout <= 32 ? 32 : (a.nout <= 64 ? 64 : 128);
    if (g_gemm_wide && a.nout > 64 && a.nout <= 96) bn = 96;
    const int64_t blocks = nrb * ((a.nout + bn - 1) / bn);
    if (bn == 32 || (blocks < 256 && nrb * ((a.nout + 31) / 32) <= 1024)) return 32;
    return bn;
}

// split-K tiles for grids of 128-row tiles that would not fill the CUs
static bool use_splitk(int mode, const GemmArgs &a)
{
    if (!g_gemm_splitk || g_splitk_suppressed || mode == GEMM_F32 || mode == GEMM_F64 || a.K1 % BK != 0 || a.K2 % BK != 0) return false;
    const int64_t nrb = (a.rows + BM - 1) / BM;
    return nrb * ((a.nout + 31) / 32) < 256;
}

static int64_t splitk_grid(const GemmArgs &a) { return ((a.rows + 31) / 32) * ((a.nout + 31) / 32); }

template <int MODE>
static void launch_splitk_mode(const GemmArgs &a, const GemmArgs *a1, hipStream_t st)
{
    const int64_t g0 = splitk_grid(a);
    if (a1) hipLaunchKernelGGL((k_gemm_splitk2<MODE>), dim3((unsigned)(g0 + splitk_grid(*a1))), dim3(256), 0, st, a,
                               *a1, g0);
    else hipLaunchKernelGGL((k_gemm_splitk<MODE>), dim3((unsigned)g0), dim3(256), 0, st, a);
}

static void launch_splitk(int mode, const GemmArgs &a, const GemmArgs *a1, hipStream_t st)
{
    with_split_mode(mode, [&](auto m) { launch_splitk_mode<decltype(m)::value>(a, a1, st); });
}

static void launch_mfma(int mode, const GemmArgs &a, const GemmArgs *a1, hipStream_t st)
{
    if (use_splitk(mode, a) && (!a1 || use_splitk(mode, *a1))) {
        launch_splitk(mode, a, a1, st);
        return;
    }
    switch (pick_bn(a)) {
    case 32: launch_bn<32>(mode, a, a1, st); break;
    case 64: launch_bn<64>(mode, a, a1, st); break;
    case 96: launch_bn<96>(mode, a, a1, st); break;
    default: launch_bn<128>(mode, a, a1, st); break;
    }
}

hipError_t launch_gemm(int mode, const GemmArgs &a, hipStream_t st)
{
    if (a.rows <= 0 || a.nout <= 0) return hipSuccess;
    if (mode == GEMM_F64) {
        dim3 grid((unsigned)((a.rows + 63) / 64), (unsigned)((a.nout + 63) / 64));
        hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, st, a);
    } else {
        launch_mfma(mode, a, nullptr, st);
    }
    // peek, so that an earlier launch's error is still there for the caller's final check
    return hipPeekAtLastError();
}

hipError_t launch_gemm2(int mode, const GemmArgs &a0, const GemmArgs &a1, hipStream_t st)
{
    const bool e0 = a0.rows <= 0 || a0.nout <= 0, e1 = a1.rows <= 0 || a1.nout <= 0;
    if (mode == GEMM_F64 || e0 || e1 || pick_bn(a0) != pick_bn(a1) || use_splitk(mode, a0) != use_splitk(mode, a1)) {
        if (!e0) (void)launch_gemm(mode, a0, st);
        if (!e1) (void)launch_gemm(mode, a1, st);
        return hipPeekAtLastError();
    }
    launch_mfma(mode, a0, &a1, st);
    return hipPeekAtLastError();
}

}  // namespace fn
