// fn_layer.hip -- one one-electron stream layer (FermiNet Model section of the
// paper) as a single kernel:
//   z = [h_i | g_i_up | g_i_dn] V_h + P_walker + b (value row),
//   h^{l+1} = tanh(z) (+ h^l)
// in forward-Laplacian form: value row y = tanh(z_0), tangent rows
// (1 - y^2) dz_c, Laplacian row (1 - y^2) lap z - 2 y (1 - y^2) sum_c dz_c^2.
//
// Tiles: 128 rows x 128 columns per 256-thread workgroup; each wave64 owns a
// 64 x 64 quarter as 4 x 4 blocks of 16 x 16 MFMA accumulators.  Operand
// tiles of 32 reduction steps go through two LDS stages (one barrier per
// step); split-BF16 operand fragments are loaded once and reused by every
// product of parts.  Each electron owns TP rows (TP = 1 value only, or 16 /
// 32 / 64), so an electron never straddles a wave's 64 rows.  The epilogue
// runs on the accumulators in registers: the sum of the squared tangent rows
// of an electron is reduced across the four lane groups of a 16-row block
// with cross-lane shuffles, and the value and Laplacian rows are broadcast
// the same way.  Output widths up to 256 columns (two halves).
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

namespace {

__device__ inline uint32_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <int NP>
__device__ inline void split(float x, uint32_t (&h)[NP])
{
    float r = x;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        h[q] = bf16_bits(r);
        r = r - __uint_as_float(h[q] << 16);
    }
}

constexpr int LBM = 128, LBN = 128, LBK = 32;
constexpr int LDH = LBK + 8;
constexpr int LDF = LBK + 4;

}  // namespace

// Block order: the two 128-column halves of one 128-row block get block ids
// that differ by 8, so that (with workgroups dealt to the eight XCDs in turn)
// both halves run on the same XCD and the second reads the rows from L2.
__device__ inline void tile_of(int b, int &rb, int &cb)
{
    const int hi = b >> 4, rem = b & 15;
    cb = rem >> 3;
    rb = hi * 8 + (rem & 7);
}

template <int MODE, int TP>
__global__ __launch_bounds__(256) void k_stream_layer(LayerArgs a)
{
    constexpr bool F32 = MODE == GEMM_F32;
    constexpr int NP = MODE == GEMM_BF16 ? 1 : (MODE == GEMM_BF16X3 ? 2 : (MODE == GEMM_BF16X6 ? 3 : 1));
    // two LDS stages: stage s holds A then B
    constexpr int ASZ = F32 ? LBM * LDF * 4 : NP * LBM * LDH * 2;
    constexpr int BSZ = F32 ? LBN * LDF * 4 : NP * LBN * LDH * 2;
    __shared__ __attribute__((aligned(16))) unsigned char smem[2 * (ASZ + BSZ)];

    int rb, cb;
    tile_of(blockIdx.x, rb, cb);
    const int64_t m0 = (int64_t)rb * LBM;
    const int n0 = cb * LBN;
    if (m0 >= a.rows || n0 >= a.W1p) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int ktiles = (a.K1 + a.K2) / LBK;
    const float *__restrict__ A1 = a.A1;
    const float *__restrict__ A2 = a.A2;

    // A tile: 4 float4 per thread (row f >> 3, columns 4 (f & 7));
    // B tile: F32 4 float4 (row f >> 3), BF16 2 uint4 per part (row f >> 2)
    int64_t arow[4];
    bool aval[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        arow[v] = m0 + ((tid + 256 * v) >> 3);
        aval[v] = arow[v] < a.rows;
    }
    float4 ra[4];
    uint4 rwh[F32 ? 1 : 2 * NP];
    float4 rwf[F32 ? 4 : 1];

    auto load_tile = [&](int kt) {
        const int kb = kt * LBK;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int f = tid + 256 * v;
            const int k = kb + 4 * (f & 7);
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (aval[v]) val = *(const float4 *)(k < a.K1 ? A1 + arow[v] * a.lda1 + k : A2 + arow[v] * a.lda2 + (k - a.K1));
            ra[v] = val;
        }
        if constexpr (F32) {
            const float *W = (const float *)a.W;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int f = tid + 256 * v;
                const int o = n0 + (f >> 3);
                rwf[v] = o < a.nout ? *(const float4 *)(W + (int64_t)o * a.ldw + kb + 4 * (f & 7))
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
            const uint16_t *W = (const uint16_t *)a.W;
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    const int f = tid + 256 * v;
                    const int o = n0 + (f >> 2);
                    rwh[q * 2 + v] = o < a.nout ? *(const uint4 *)(W + (int64_t)q * a.wpart + (int64_t)o * a.ldw + kb +
                                                                   8 * (f & 3))
                                                : make_uint4(0, 0, 0, 0);
                }
        }
    };
    auto store_tile = [&](int stage) {
        unsigned char *base = smem + stage * (ASZ + BSZ);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int f = tid + 256 * v;
            const int r = f >> 3, k = 4 * (f & 7);
            const float4 x = ra[v];
            if constexpr (F32) {
                *(float4 *)((float *)base + r * LDF + k) = x;
            } else {
                uint32_t h0[NP], h1[NP], h2[NP], h3[NP];
                split<NP>(x.x, h0);
                split<NP>(x.y, h1);
                split<NP>(x.z, h2);
                split<NP>(x.w, h3);
#pragma unroll
                for (int q = 0; q < NP; ++q)
                    *(uint2 *)((uint16_t *)base + q * LBM * LDH + r * LDH + k) =
                        make_uint2(h0[q] | (h1[q] << 16), h2[q] | (h3[q] << 16));
            }
        }
        if constexpr (F32) {
            float *sB = (float *)(base + ASZ);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int f = tid + 256 * v;
                *(float4 *)&sB[(f >> 3) * LDF + 4 * (f & 7)] = rwf[v];
            }
        } else {
            uint16_t *sB = (uint16_t *)(base + ASZ);
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    const int f = tid + 256 * v;
                    *(uint4 *)&sB[q * LBN * LDH + (f >> 2) * LDH + 8 * (f & 3)] = rwh[q * 2 + v];
                }
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (ktiles > 0) {
        load_tile(0);
        store_tile(0);
    }
    for (int kt = 0; kt < ktiles; ++kt) {
        __syncthreads();                         // stage kt & 1 is complete, stage (kt + 1) & 1 is free
        if (kt + 1 < ktiles) load_tile(kt + 1);
        const unsigned char *base = smem + (kt & 1) * (ASZ + BSZ);
        const int ar = wm * 64 + (lane & 15), br = wn * 64 + (lane & 15);
        if constexpr (F32) {
            const float *sA = (const float *)base, *sB = (const float *)(base + ASZ);
#pragma unroll
            for (int kk = 0; kk < LBK / 4; ++kk) {
                float fa[4], fb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) fa[i] = sA[(ar + 16 * i) * LDF + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int j = 0; j < 4; ++j) fb[j] = sB[(br + 16 * j) * LDF + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        } else {
            const uint16_t *sA = (const uint16_t *)base, *sB = (const uint16_t *)(base + ASZ);
            const int ko = 8 * (lane >> 4);
            bf16x8 ha[NP][4], hb[NP][4];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ha[q][i] = *(const bf16x8 *)&sA[q * LBM * LDH + (ar + 16 * i) * LDH + ko];
#pragma unroll
                for (int j = 0; j < 4; ++j) hb[q][j] = *(const bf16x8 *)&sB[q * LBN * LDH + (br + 16 * j) * LDH + ko];
            }
            // products of parts (pa, pb) with pa + pb < NP, smallest first
#pragma unroll
            for (int sum = NP - 1; sum >= 0; --sum)
#pragma unroll
                for (int pa = 0; pa <= sum; ++pa)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[pa][i], hb[sum - pa][j], acc[i][j],
                                                                                0, 0, 0);
        }
        if (kt + 1 < ktiles) store_tile((kt + 1) & 1);
    }

    // ---- epilogue: accumulator (i, j)[e] is row 64 wm + 16 i + 4 (lane >> 4) + e,
    //      column n0 + 64 wn + 16 j + (lane & 15)
    const int lg = lane >> 4, lc = lane & 15;
    const float *__restrict__ Pw = a.Pw;
    const float *__restrict__ bias = a.bias;
    const float *__restrict__ Hin = a.A1;
    float *__restrict__ Hout = a.Hout;
    const int n3 = a.n3;
    const int64_t mw = m0 + 64 * wm;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn * 64 + 16 * j + lc;
        if (col >= a.W1p) continue;
        const bool real = col < a.w1;
        const float bcol = real ? bias[col] : 0.f;
        if constexpr (TP == 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t R = mw + 16 * i + 4 * lg + e;
                    if (R >= a.rows) continue;
                    float y = 0.f;
                    if (real) {
                        const int64_t w = R / a.N;
                        y = tanhf(acc[i][j][e] + Pw[w * a.w1 + col] + bcol);
                        if (a.resid) y += Hin[R * a.lda1 + col];
                    }
                    Hout[R * a.ldh_out + col] = y;
                }
        } else {
            constexpr int IB = TP / 16;                 // 16-row blocks per electron
            const int tl = n3 + 1;                      // Laplacian row of an electron
            const int ibl = tl >> 4, lgl = (tl >> 2) & 3, el = tl & 3;
#pragma unroll
            for (int ib0 = 0; ib0 < 4; ib0 += IB) {
                const int64_t Rb = mw + 16 * ib0;       // first row of this electron
                if (Rb >= a.rows) continue;
                const int64_t E = Rb / TP;
                const int64_t w = E / a.N;
                const float *pw = Pw + (w * TP) * (int64_t)a.w1 + col;
                float z[IB][4];
                float src = 0.f, cand = 0.f;
#pragma unroll
                for (int q = 0; q < IB; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int t = 16 * q + 4 * lg + e;
                        float v = acc[ib0 + q][j][e];
                        if (real) v += pw[(int64_t)t * a.w1] + (t == 0 ? bcol : 0.f);
                        z[q][e] = v;
                        if (t >= 1 && t <= n3) src += v * v;
                        if (q == ibl && e == el) cand = v;
                    }
                src += __shfl_xor(src, 16, 64);
                src += __shfl_xor(src, 32, 64);
                const float z0 = __shfl(z[0][0], lc, 64);
                const float zl = __shfl(cand, 16 * lgl + lc, 64);
                const float y0 = tanhf(z0);
                const float d = 1.f - y0 * y0;
#pragma unroll
                for (int q = 0; q < IB; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int t = 16 * q + 4 * lg + e;
                        const int64_t R = Rb + t;
                        float y = 0.f;
                        if (real && t <= tl) {
                            y = t == 0 ? y0 : (t < tl ? d * z[q][e] : d * zl - 2.f * y0 * d * src);
                            if (a.resid) y += Hin[R * a.lda1 + col];
                        }
                        Hout[R * a.ldh_out + col] = y;
                    }
            }
        }
    }
}

// The fused layer is kept out of the default path until its operand pipeline
// hides the load latency at this reduction depth (K = 320): measured slower
// than the separate product + epilogue on LiH.
bool g_use_fused_layer = false;

bool stream_layer_supported(int mode, int TR, int W1p)
{
    return g_use_fused_layer && mode != GEMM_F64 && W1p <= 2 * LBN && (TR == 1 || TR == 16 || TR == 32 || TR == 64);
}

template <int MODE>
static void launch_mode(const LayerArgs &a, int TR, hipStream_t st)
{
    const int64_t rblocks = (a.rows + LBM - 1) / LBM;
    dim3 grid((unsigned)(((rblocks + 7) / 8) * 16));
    switch (TR) {
    case 1: hipLaunchKernelGGL((k_stream_layer<MODE, 1>), grid, dim3(256), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_stream_layer<MODE, 16>), grid, dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_stream_layer<MODE, 32>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((k_stream_layer<MODE, 64>), grid, dim3(256), 0, st, a); break;
    }
}

void launch_stream_layer(int mode, const LayerArgs &a, int TR, hipStream_t st)
{
    if (a.rows <= 0) return;
    switch (mode) {
    case GEMM_F32: launch_mode<GEMM_F32>(a, TR, st); break;
    case GEMM_BF16: launch_mode<GEMM_BF16>(a, TR, st); break;
    case GEMM_BF16X3: launch_mode<GEMM_BF16X3>(a, TR, st); break;
    default: launch_mode<GEMM_BF16X6>(a, TR, st); break;
    }
}

}  // namespace fn
