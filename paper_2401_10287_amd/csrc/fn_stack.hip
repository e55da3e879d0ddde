// fn_stack.hip -- all one-electron stream layers of the forward-Laplacian
// pass (FermiNet Model section of the paper) in one kernel, for systems of
// two to four electrons (16 rows per electron: value, 3N tangents,
// Laplacian, padding), in the split-BF16 modes.
//
// A workgroup keeps the rows of W whole walkers (W N 16 <= 64, or <= 128
// rows) in LDS
// for the whole pass, so the activations never return to HBM between
// layers.  Per layer l:
//   P = [g_up | g_dn] V_g              (one 16-row block per walker; the
//                                       spin means of h are formed from LDS
//                                       as the operand fragments are read)
//   X = [h | g_i_up | g_i_dn] V_h      (rows of every (walker, electron))
//   h^{l+1} = tanh(X + P + b) (+ h^l)  with the forward-Laplacian epilogue:
//     value y = tanh(z_0), tangents (1 - y^2) z_c, Laplacian
//     (1 - y^2) z_L - 2 y (1 - y^2) sum_c z_c^2.
// Each of the four waves owns 64 of the 256 output columns for all rows:
// 16 x 16 accumulator blocks (row block = one electron's 16 rows), so the
// epilogue of a column runs in registers (the value row's tanh broadcast and
// the source sum over the tangent rows by lane exchanges).  Weights come
// from global memory (L2) straight into registers, the next reduction step's
// fragments requested before the current step's matrix instructions; the
// pair means g_i of the layer are copied into LDS beside h.
// LDS: rows x 320 floats (h: 256 columns, g_i: 64), 16-byte chunks
// XOR-swizzled by the row's low three bits.
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

namespace {

constexpr int SW = 320;                      // floats per LDS row: h (256) | g_i (64)

// float index of element (row r, column k) in the swizzled LDS tile
__device__ inline int sidx(int r, int k) { return r * SW + 4 * ((k >> 2) ^ (r & 7)) + (k & 3); }

__device__ inline float4 ld4(const float *s, int r, int k) { return *(const float4 *)(s + sidx(r, k)); }

}  // namespace

// Raw weight registers of one reduction step: the BF16 parts as packed, or
// (WF) the FP32 values, split into parts in registers when used -- one FP32
// copy of every layer's weights stays in L2 where three BF16 parts do not.
template <int NP, bool WF> struct WRegs { uint4 v[NP][4]; };
template <int NP> struct WRegs<NP, true> { float4 v[4][2]; };

// W walkers per workgroup; PF: the next reduction step's weight fragments
// are requested before the current step's matrix instructions (one wave
// per SIMD), else two workgroups share each CU and hide each other's loads
template <int NP, int NE, int W, bool PF, bool WF>
__global__ __launch_bounds__(256, PF ? 1 : 2) void k_stack_fl(StackArgs a)
{
    constexpr int RB = W * NE;                   // 16-row blocks, one per (walker, electron)
    constexpr int ROWS = RB * 16;
    __shared__ __attribute__((aligned(16))) float sH[ROWS * SW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, kq = lane >> 4;
    const int64_t w0 = (int64_t)blockIdx.x * W;
    const int nw = (int)(a.B - w0 < W ? a.B - w0 : W);
    const int col0 = 64 * wave;
    const int n3 = a.n3, tl = n3 + 1;
    const int nu = a.nu, nd = NE - a.nu;
    const float inv_u = nu ? 1.f / (float)nu : 0.f, inv_d = nd ? 1.f / (float)nd : 0.f;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);

    // layer 0's input: the features of this workgroup's walkers
    {
        const int c4n = a.HW[0] / 4;
        for (int q = tid; q < ROWS * c4n; q += 256) {
            const int r = q / c4n, c4 = q - r * c4n;
            float4 v = zero4;
            if (r / (NE * 16) < nw) v = *(const float4 *)(a.H0 + (w0 * NE * 16 + r) * a.ldh + 4 * c4);
            *(float4 *)(sH + sidx(r, 4 * c4)) = v;
        }
    }

    for (int l = 0; l < a.L; ++l) {
        const int HW = a.HW[l], GW = a.GW[l];
        const int kx = (HW + GW) >> 5, kg = (2 * HW) >> 5;
        const uint16_t *__restrict__ Wx = a.Wx[l];
        const uint16_t *__restrict__ Wg = a.Wg[l];
        const int64_t px = a.wxpart[l], pg = a.wgpart[l];
        const int ldx = HW + GW, ldgw = 2 * HW;
        // the layer's pair means into LDS columns 256 .. 256 + GW (padding rows
        // of an electron and rows of absent walkers are zero)
        {
            const float *__restrict__ GI = a.GI + (int64_t)l * a.gi_stride;
            const int c4n = GW / 4;
            for (int q = tid; q < ROWS * c4n; q += 256) {
                const int r = q / c4n, c4 = q - r * c4n;
                float4 v = zero4;
                if (r / (NE * 16) < nw && (r & 15) <= tl) v = *(const float4 *)(GI + (w0 * NE * 16 + r) * a.ldgi + 4 * c4);
                *(float4 *)(sH + sidx(r, 256 + 4 * c4)) = v;
            }
        }
        __syncthreads();

        f32x4 acc[RB][4], pac[W][4];

        // weight fragment of column block j, part q, reduction step kb: row
        // col0 + 16 j + li, elements kb + 8 kq .. + 7
        int64_t wrow[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) wrow[j] = (int64_t)(col0 + 16 * j + li);
        const float *__restrict__ Wx32 = a.Wx32[l];
        const float *__restrict__ Wg32 = a.Wg32[l];
        typedef WRegs<NP, WF> WR;
        auto load_w = [&](const uint16_t *W16, const float *W32, int64_t part, int ld, int kt, WR &B) {
            if constexpr (WF) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float *src = W32 + wrow[j] * ld + 32 * kt + 8 * kq;
                    B.v[j][0] = *(const float4 *)src;
                    B.v[j][1] = *(const float4 *)(src + 4);
                }
            } else {
#pragma unroll
                for (int q = 0; q < NP; ++q)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        B.v[q][j] = *(const uint4 *)(W16 + q * part + wrow[j] * ld + 32 * kt + 8 * kq);
            }
        };
        auto load_wx = [&](int kt, WR &B) { load_w(Wx, Wx32, px, ldx, kt, B); };
        auto load_wg = [&](int kt, WR &B) { load_w(Wg, Wg32, pg, ldgw, kt, B); };
        // the BF16 parts of a step's weight fragments
        auto parts = [&](const WR &B, bf16x8 (&hb)[NP][4]) {
            if constexpr (WF) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    bf16x8 p[NP];
                    split_fragment<NP>(B.v[j][0], B.v[j][1], p);
#pragma unroll
                    for (int q = 0; q < NP; ++q) hb[q][j] = p[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < NP; ++q)
#pragma unroll
                    for (int j = 0; j < 4; ++j) hb[q][j] = __builtin_bit_cast(bf16x8, B.v[q][j]);
            }
        };
        WR cur, nxt;

        // ---- P = [g_up | g_dn] V_g, one row block per walker (rows t = li)
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
            for (int j = 0; j < 4; ++j) pac[w][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        // the mean-field steps carry a quarter of the matrix work per weight
        // fragment: the next step's fragments are always requested first
        auto p_step = [&](int kt, const WR &B) {
            const int kb = 32 * kt;
            const bool dn = kb >= HW;
            const int kc = (dn ? kb - HW : kb) + 8 * kq;
            const int e0 = dn ? nu : 0, e1 = dn ? NE : nu;
            const float sc = dn ? inv_d : inv_u;
            bf16x8 hb[NP][4];
            parts(B, hb);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                float4 s0 = zero4, s1 = zero4;
                for (int e = e0; e < e1; ++e) {       // electrons of the spin, in order
                    const int r = 16 * (w * NE + e) + li;
                    const float4 x0 = ld4(sH, r, kc), x1 = ld4(sH, r, kc + 4);
                    s0 = make_float4(s0.x + x0.x, s0.y + x0.y, s0.z + x0.z, s0.w + x0.w);
                    s1 = make_float4(s1.x + x1.x, s1.y + x1.y, s1.z + x1.z, s1.w + x1.w);
                }
                s0 = make_float4(s0.x * sc, s0.y * sc, s0.z * sc, s0.w * sc);
                s1 = make_float4(s1.x * sc, s1.y * sc, s1.z * sc, s1.w * sc);
                bf16x8 ha[NP];
                split_fragment<NP>(s0, s1, ha);
#pragma unroll
                for (int sum = NP - 1; sum >= 0; --sum)
#pragma unroll
                    for (int pa = 0; pa <= sum; ++pa)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            pac[w][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[pa], hb[sum - pa][j], pac[w][j],
                                                                                0, 0, 0);
            }
        };
        load_wg(0, cur);
        for (int kt = 0; kt < kg; ++kt) {
            if (kt + 1 < kg) load_wg(kt + 1, nxt);
            p_step(kt, cur);
            if (kt + 1 < kg) cur = nxt;
        }

        // ---- X = [h | g_i] V_h over all (walker, electron) row blocks
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[rb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (PF) load_wx(0, cur);
        for (int kt = 0; kt < kx; ++kt) {
            if constexpr (PF) {
                if (kt + 1 < kx) load_wx(kt + 1, nxt);
            } else {
                load_wx(kt, cur);
            }
            const int kb = 32 * kt;
            const int kc = kb < HW ? kb + 8 * kq : 256 + (kb - HW) + 8 * kq;   // LDS column of this lane's fragment
            bf16x8 hb[NP][4];
            parts(cur, hb);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int r = 16 * rb + li;
                const float4 x0 = ld4(sH, r, kc), x1 = ld4(sH, r, kc + 4);
                bf16x8 ha[NP];
                split_fragment<NP>(x0, x1, ha);
#pragma unroll
                for (int sum = NP - 1; sum >= 0; --sum)
#pragma unroll
                    for (int pa = 0; pa <= sum; ++pa)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[pa], hb[sum - pa][j], acc[rb][j],
                                                                                 0, 0, 0);
            }
            if constexpr (PF) {
                if (kt + 1 < kx) cur = nxt;
            }
        }

        // every wave has read every column of h^l: the columns can be replaced
        __syncthreads();

        // ---- epilogue: rows t = 4 kq + i of each electron, column col0 + 16 j + li
        const float *__restrict__ bias = a.bias[l];
        const bool resid = l >= 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = col0 + 16 * j + li;
            const float bc = bias[col];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int w = rb / NE;
                float z[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    z[i] = acc[rb][j][i] + pac[w][j][i];
                    if (kq == 0 && i == 0) z[i] = z[i] + bc;        // (X + P) + b on the value row
                }
                const float z0 = __shfl(z[0], li, 64);              // value row (lane li, i = 0)
                float src = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int t = 4 * kq + i;
                    if (t >= 1 && t <= n3) src += z[i] * z[i];
                }
                src += __shfl_xor(src, 16, 64);
                src += __shfl_xor(src, 32, 64);
                const float y0 = tanhf(z0);
                const float dd = 1.f - y0 * y0;
                const float lapsrc = 2.f * y0 * dd * src;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int t = 4 * kq + i;
                    const int r = 16 * rb + t;
                    float y = 0.f;
                    if (t == 0) y = y0;
                    else if (t < tl) y = dd * z[i];
                    else if (t == tl) y = dd * z[i] - lapsrc;
                    if (t <= tl && resid) y = y + sH[sidx(r, col)];
                    sH[sidx(r, col)] = y;
                }
            }
        }
        __syncthreads();
    }

    // h^L of the live rows to global memory for the orbital head
    for (int q = tid; q < ROWS * 64; q += 256) {
        const int r = q >> 6, c4 = q & 63;
        if (r / (NE * 16) >= nw || (r & 15) > tl) continue;
        *(float4 *)(a.Hout + (w0 * NE * 16 + r) * a.ldh + 4 * c4) = *(const float4 *)(sH + sidx(r, 4 * c4));
    }
}

// 0: never; 1 (default): the one-pass BF16 mode, where the stacked kernel
// is the faster one; 2: every split-BF16 mode (the split modes measure
// slower stacked: each wave splits every activation fragment it reads, and
// the register budget leaves no room to hide load latency; the six-product
// split reads FP32 weights, split in registers, so that every layer's
// weights stay in L2 -- three BF16 parts of all four layers did not)
int g_use_stack = 1;

bool stack_supported(int mode, int N, int TR, int w1, int L)
{
    const bool on = g_use_stack == 2 ? (mode == GEMM_BF16 || mode == GEMM_BF16X3 || mode == GEMM_BF16X6)
                                     : (g_use_stack == 1 && mode == GEMM_BF16);
    return on && TR == 16 && N >= 2 && N <= 4 && w1 == 256 && L <= FN_MAX_LAYERS;
}

// workgroup shape (tuning switch "stack_shape"): 0 = 64 rows (N = 4: one
// walker), two workgroups per CU; 1 = 64 rows, one per CU with the next
// step's weights prefetched; 2 = 128 rows, prefetched
int g_stack_shape = 0;

template <int NP, int NE, bool WF>
static void launch_ne(const StackArgs &a, hipStream_t st)
{
    constexpr int W1 = 4 / NE, W2 = NE == 3 ? 2 : 8 / NE;
    const dim3 b(256);
    if (g_stack_shape == 2)
        hipLaunchKernelGGL((k_stack_fl<NP, NE, W2, true, WF>), dim3((unsigned)((a.B + W2 - 1) / W2)), b, 0, st, a);
    else if (g_stack_shape == 1)
        hipLaunchKernelGGL((k_stack_fl<NP, NE, W1, true, WF>), dim3((unsigned)((a.B + W1 - 1) / W1)), b, 0, st, a);
    else
        hipLaunchKernelGGL((k_stack_fl<NP, NE, W1, false, WF>), dim3((unsigned)((a.B + W1 - 1) / W1)), b, 0, st, a);
}

template <int NP, bool WF>
static void launch_np(const StackArgs &a, int N, hipStream_t st)
{
    switch (N) {
    case 2: launch_ne<NP, 2, WF>(a, st); break;
    case 3: launch_ne<NP, 3, WF>(a, st); break;
    default: launch_ne<NP, 4, WF>(a, st); break;
    }
}

void launch_stack(int mode, const StackArgs &a, int N, hipStream_t st)
{
    if (a.B <= 0) return;
    switch (mode) {
    case GEMM_BF16: launch_np<1, false>(a, N, st); break;
    case GEMM_BF16X3: launch_np<2, false>(a, N, st); break;
    default:
        if (a.Wx32[0]) launch_np<3, true>(a, N, st);
        else launch_np<3, false>(a, N, st);
        break;
    }
}

}  // namespace fn
