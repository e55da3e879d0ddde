// fn_stackr.hip -- every one-electron stream layer of a forward-Laplacian
// pass (FermiNet Model section of the paper) in one kernel with the
// activations held in registers, for walkers of four electrons, two of each
// spin (16 rows per electron: value, 12 tangents, Laplacian, padding),
// w1 = 256, in the modes whose layer weights are one BF16 part (activations
// split into NA exact-or-rounded BF16 parts).
//
// Workgroup: four waves and two walkers.  Wave q owns the two electrons of
// spin q & 1 of walker q >> 1 (electrons are stored spin-up first), all 256
// output columns of their 32 rows.  Every product runs transposed,
//   D^T = W^T X^T,
// so the weight fragments (rows = output columns) are the matrix
// instruction's A operand, read from an LDS ring that the four waves share,
// and the activations are the B operand, taken from the wave's own
// registers.  Accumulator ("D") layout: lane (t = lane % 16, og = lane / 16)
// of block c holds output columns 16 c + 4 og + e, e = 0..3, of row t of an
// electron.  The B operand of reduction step s (input columns 32 s + 8 kg ..
// + 7 of row t in lane (t, kg)) is formed from blocks 2 s and 2 s + 1 of the
// previous layer's output by one 32-lane and one 16-lane swap per element.
//
// Per layer l:
//   A phase: P_spin = g_spin V_g^spin over the wave's own spin (g = mean of
//            its two electrons' h), one 16-row block, then exchanged: the
//            spin-up wave stores its partial, the spin-down wave adds its own
//            (P = P_up + P_dn, the same in both waves).
//   B phase: X = [h | g_i_up | g_i_dn] V_h for both electrons (the pair
//            means g_i come through the ring as well, each wave its own rows).
//   epilogue in registers: z = (X + P) + b, value y = tanh(z_0) (formed once
//            per column through a per-wave LDS scratch), tangents (1 - y^2) z_c,
//            Laplacian (1 - y^2) z_L - 2 y (1 - y^2) sum_c z_c^2 (the source sum
//            over the 16 lanes of a row group by DPP butterflies), residual.
// Weights stream through the ring as 16 KB tiles (256 output rows x 32
// reduction columns) by direct global-to-LDS copies, several tiles ahead;
// each step waits only for its own tiles.  Only the features, the pair
// means and h^L touch HBM.
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

namespace {

constexpr int RT = 6;                 // ring tiles of 16 KB
constexpr int TILE = 16384;
constexpr int CPT = 4;                // 16-byte copies per lane per tile

// until at most CPT * n vector-memory operations of this wave are
// outstanding (n tiles still in flight; waiting for fewer is always safe)
__device__ inline void wait_tiles(int n)
{
#define FN_WVM(k) \
    case k: __builtin_amdgcn_s_waitcnt(0x0F70 | ((CPT * (k)) & 15) | (((CPT * (k)) >> 4) << 14)); break;
    switch (n < 0 ? 0 : (n > RT ? RT : n)) {
        FN_WVM(0) FN_WVM(1) FN_WVM(2) FN_WVM(3) FN_WVM(4) FN_WVM(5) FN_WVM(6)
    }
#undef FN_WVM
}
static_assert(RT <= 6 && CPT * RT < 64, "wait_tiles cases");

// workgroup barrier that leaves outstanding global loads alone: this wave's
// LDS operations complete first, and no memory access moves across it
__device__ inline void ring_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt untouched
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// buffer resource over n bytes from base (wave-uniform); loads past n read zero
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, 0x00020000);
}
// 16 bytes at byte offset voff of the buffer into lds + 16 * lane (lds: the
// wave's 1 KB block)
__device__ inline void copy16_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, void *lds)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)lds, 16, voff, 0, 0, 0);
}

// D layout -> B operand: blocks x0 = 2 s, x1 = 2 s + 1 of one electron's
// rows give the eight columns 32 s + 8 kg + m of row t (m = e in lo, 4 + e in hi)
__device__ inline void d_to_b(const f32x4 &x0, const f32x4 &x1, float4 &lo, float4 &hi)
{
    float l[4], h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0[e]), __float_as_uint(x1[e]), false, false);
        const auto q = __builtin_amdgcn_permlane16_swap(r[0], r[1], false, false);
        l[e] = __uint_as_float(q[0]);
        h[e] = __uint_as_float(q[1]);
    }
    lo = make_float4(l[0], l[1], l[2], l[3]);
    hi = make_float4(h[0], h[1], h[2], h[3]);
}

// sum over the 16 lanes of a row group, the same bits in every lane
__device__ inline float sum16(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
    return v;
}

__device__ inline float4 mask4r(float4 x, bool keep) { return keep ? x : make_float4(0.f, 0.f, 0.f, 0.f); }

}  // namespace

template <int NA>
__global__ __launch_bounds__(256, 1) void k_stack_regs(StackArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char ring[RT * TILE];
    __shared__ __attribute__((aligned(16))) f32x4 pex[2][16][64];     // P of each walker, D layout
    __shared__ __attribute__((aligned(16))) float vsc[4][2][512];     // per wave: value rows -> tanh, 1 - tanh^2
    __shared__ __attribute__((aligned(16))) float sbias[FN_MAX_LAYERS][256];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int t = lane & 15, og = lane >> 4;
    const int wl = wave >> 1, sig = wave & 1;
    const int64_t w = 2 * (int64_t)blockIdx.x + wl;
    const bool live = w < a.B;
    const int64_t wc = live ? w : a.B - 1;           // loads of an absent walker read a valid one
    const int n3 = a.n3, tl = n3 + 1;
    const bool trow = t <= tl;                        // rows past the Laplacian row are padding
    const float fval = t == 0 ? 1.f : 0.f;            // value row
    const float ftan = t >= 1 && t <= n3 ? 1.f : 0.f; // tangent rows
    const float flap = t == tl ? 1.f : 0.f;           // Laplacian row
    const int64_t row0 = (wc * 4 + 2 * sig) * 16;    // first row of this wave's electrons
    int64_t row[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) row[rb] = row0 + 16 * rb + t;

    // ---- ring tiles, in consumption order, per layer: for each spin-mean
    //      step the V_g tiles of both spins; for each input step of h the
    //      V_h tile; for each pair-mean step the V_h tile and then the pair
    //      means of every wave's rows (4 KB per wave, rows chunk-swizzled)
    auto layer_tiles = [&](int l) { return 2 * (a.HW[l] >> 5) + (a.HW[l] >> 5) + 2 * (a.GW[l] >> 5); };
    int NT = 0;
    for (int l = 0; l < a.L; ++l) NT += layer_tiles(l);
    int il = 0, iu = 0;                              // layer and in-layer index of the next tile to issue
    auto issue = [&](int T) {
        const int l = il, u = iu, nA2 = 2 * (a.HW[l] >> 5), nH = a.HW[l] >> 5;
        if (++iu == layer_tiles(il)) {
            iu = 0;
            ++il;
        }
        unsigned char *slot = ring + (T % RT) * TILE;
        if (u >= nA2 + nH && ((u - nA2 - nH) & 1)) {
            // pair means, step g: rows 8 j + lane / 8 of this wave's 32,
            // 16-byte chunk c of the row stored at slot c ^ (row & 7)
            const int g = (u - nA2 - nH) >> 1;
            const float *base = a.GI + (int64_t)l * a.gi_stride + row0 * a.ldgi + 32 * g;
            const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(base, (uint32_t)(32 * a.ldgi * 4));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 8 * j + (lane >> 3);
                copy16_buf(rs, (uint32_t)(r * a.ldgi * 4 + 16 * ((lane & 7) ^ (r & 7))), slot + wave * 4096 + j * 1024);
            }
            return;
        }
        const uint16_t *W;
        int ld, k0;
        if (u < nA2) {
            W = a.Wg[l];
            ld = 2 * a.HW[l];
            k0 = (u & 1) * a.HW[l] + 32 * (u >> 1);
        } else {
            const int v = u - nA2;
            W = a.Wx[l];
            ld = a.HW[l] + a.GW[l];
            k0 = 32 * (v < nH ? v : nH + ((v - nH) >> 1));
        }
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(W + k0, (uint32_t)(256 * ld * 2));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = 4 * wave + j;
            const int o = 16 * b + (lane >> 2);
            copy16_buf(rs, (uint32_t)(o * ld * 2 + 16 * lds_chunk(o, lane & 3)), slot + b * 1024);
        }
    };
    // every layer's bias into LDS before any copy is in flight (read after
    // the barriers of the first steps)
    for (int q = tid; q < a.L * 64; q += 256) *(float4 *)&sbias[q >> 6][4 * (q & 63)] = *(const float4 *)(a.bias[q >> 6] + 4 * (q & 63));
    int issued = 0, first = 0;
    // every lane has landed the tiles before `need`, then the workgroup
    // agrees; tiles that no step before `first` still reads are refilled
    auto step_sync = [&](int need) {
        wait_tiles(issued - need);
        ring_barrier();
        while (issued < NT && issued < first + RT) issue(issued++);
    };
    while (issued < NT && issued < RT) issue(issued++);

    // A fragment of output block c in a ring tile: row 16 c + t, chunk og
    const int afrag = t * 64 + 16 * lds_chunk(t, og);

    f32x4 hp[2][16];                                  // h of this layer's input (then output), D layout
    f32x4 acc[2][16];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int c = 0; c < 16; ++c) hp[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int l = 0; l < a.L; ++l) {
        const int nA = a.HW[l] >> 5, nH = nA, nG = a.GW[l] >> 5;
        const bool l0 = l == 0;

        // B operand of input step s (s < nH) of electron rb; the register
        // blocks are chosen by a switch so that the step loops stay loops
        auto h_operand = [&](int s, int rb, float4 &lo, float4 &hi) {
            if (l0) {
                const float *p = a.H0 + row[rb] * a.ldh + 32 * s + 8 * og;
                lo = mask4r(*(const float4 *)p, trow);
                hi = mask4r(*(const float4 *)(p + 4), trow);
                return;
            }
#define FN_HB(k) \
    case k: d_to_b(hp[rb][2 * (k)], hp[rb][2 * (k) + 1], lo, hi); break;
            switch (s) { FN_HB(0) FN_HB(1) FN_HB(2) FN_HB(3) FN_HB(4) FN_HB(5) FN_HB(6) default: FN_HB(7) }
#undef FN_HB
        };

        // ---- A phase: this wave's spin-mean partial of the mean-field product
        f32x4 pm[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) pm[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int s = 0; s < nA; ++s) {
            step_sync(first + 2);
            float4 l0v, h0v, l1v, h1v;
            h_operand(s, 0, l0v, h0v);
            h_operand(s, 1, l1v, h1v);
            // mean of the spin's two electrons, (h_0 + h_1) / 2
            const float4 lo = make_float4((l0v.x + l1v.x) * 0.5f, (l0v.y + l1v.y) * 0.5f, (l0v.z + l1v.z) * 0.5f,
                                          (l0v.w + l1v.w) * 0.5f);
            const float4 hi = make_float4((h0v.x + h1v.x) * 0.5f, (h0v.y + h1v.y) * 0.5f, (h0v.z + h1v.z) * 0.5f,
                                          (h0v.w + h1v.w) * 0.5f);
            bf16x8 hb[NA];
            split_fragment<NA>(lo, hi, hb);
            // four column blocks at a time, the next four requested first
            const unsigned char *tile = ring + ((first + sig) % RT) * TILE + afrag;
            bf16x8 wa[4], wn[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) wa[j] = *(const bf16x8 *)(tile + j * 1024);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (g < 3) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) wn[j] = *(const bf16x8 *)(tile + (4 * g + 4 + j) * 1024);
                }
#pragma unroll
                for (int p = 0; p < NA; ++p)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        pm[4 * g + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], hb[p], pm[4 * g + j], 0, 0, 0);
                if (g < 3) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) wa[j] = wn[j];
                }
            }
            first += 2;
        }
        // the spin-up wave stores its partial; the spin-down wave adds its own
        // (P = P_up + P_dn in both)
        if (sig == 0) {
#pragma unroll
            for (int c = 0; c < 16; ++c) pex[wl][c][lane] = pm[c];
        }

        // the partner's partial is stored (before this barrier); the sum is
        // complete before the barrier of the first B step
        ring_barrier();
        if (sig == 1) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                f32x4 v = pex[wl][c][lane];
                v += pm[c];
                pex[wl][c][lane] = v;
            }
        }

        // ---- B phase: X = [h | g_i] V_h for both electrons
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int c = 0; c < 16; ++c) acc[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        // one reduction step with the operands of both electrons in hb: two
        // column blocks at a time (the next two requested first), parts
        // outermost within them (four accumulators between dependent products)
        auto b_products = [&](const bf16x8 (&hb)[2][NA]) {
            const unsigned char *tile = ring + (first % RT) * TILE + afrag;
            bf16x8 wa[2], wn[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) wa[j] = *(const bf16x8 *)(tile + j * 1024);
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                if (g < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wn[j] = *(const bf16x8 *)(tile + (2 * g + 2 + j) * 1024);
                }
#pragma unroll
                for (int p = 0; p < NA; ++p)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb)
                            acc[rb][2 * g + j] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], hb[rb][p], acc[rb][2 * g + j], 0, 0, 0);
                if (g < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
        };
        // input steps of h
#pragma unroll 1
        for (int s = 0; s < nH; ++s) {
            step_sync(first + 1);
            bf16x8 hb[2][NA];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                float4 lo, hi;
                h_operand(s, rb, lo, hi);
                split_fragment<NA>(lo, hi, hb[rb]);
            }
            b_products(hb);
            first += 1;
        }
        // pair-mean steps: the V_h tile, then this wave's pair-mean rows
#pragma unroll 1
        for (int g = 0; g < nG; ++g) {
            step_sync(first + 2);
            bf16x8 hb[2][NA];
            const unsigned char *gt = ring + ((first + 1) % RT) * TILE + wave * 4096;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const int r = 16 * rb + t;
                const float4 lo = mask4r(*(const float4 *)(gt + r * 128 + 16 * ((2 * og) ^ (r & 7))), trow);
                const float4 hi = mask4r(*(const float4 *)(gt + r * 128 + 16 * ((2 * og + 1) ^ (r & 7))), trow);
                split_fragment<NA>(lo, hi, hb[rb]);
            }
            b_products(hb);
            first += 2;
        }

        // ---- epilogue, branch-free: row roles as multipliers and selects;
        //      padding rows come out zero (their z is exactly zero)
        float *z0s = vsc[wave][0], *dds = vsc[wave][1];
        const float *bl = sbias[l];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const f32x4 P = pex[wl][c][lane];
            const float4 b4 = *(const float4 *)(bl + 16 * c + 4 * og);
            const f32x4 bv = f32x4{b4.x * fval, b4.y * fval, b4.z * fval, b4.w * fval};
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const f32x4 z = (acc[rb][c] + P) + bv;          // (X + P) + b on the value row
                acc[rb][c] = z;
                if (t == 0) *(f32x4 *)(z0s + 256 * rb + 16 * c + 4 * og) = z;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        {
            // tanh of the 512 value-row entries, eight per lane
            float4 u[2];
            u[0] = *(const float4 *)(z0s + 8 * lane);
            u[1] = *(const float4 *)(z0s + 8 * lane + 4);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const float4 y = make_float4(tanhf(u[k].x), tanhf(u[k].y), tanhf(u[k].z), tanhf(u[k].w));
                *(float4 *)(z0s + 8 * lane + 4 * k) = y;
                *(float4 *)(dds + 8 * lane + 4 * k) =
                    make_float4(1.f - y.x * y.x, 1.f - y.y * y.y, 1.f - y.z * y.z, 1.f - y.w * y.w);
            }
        }
        const float fres = l >= 1 ? 1.f : 0.f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const float4 y4 = *(const float4 *)(z0s + 256 * rb + 16 * c + 4 * og);
                const float4 d4 = *(const float4 *)(dds + 256 * rb + 16 * c + 4 * og);
                const float y0[4] = {y4.x, y4.y, y4.z, y4.w}, dd[4] = {d4.x, d4.y, d4.z, d4.w};
                const f32x4 z = acc[rb][c];
                f32x4 y;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float src = sum16((z[e] * z[e]) * ftan);      // over the tangent rows
                    const float lapc = (2.f * y0[e] * dd[e]) * flap;     // Laplacian row only
                    const float v = dd[e] * z[e] - lapc * src;
                    y[e] = (t == 0 ? y0[e] : v) + fres * hp[rb][c][e];
                }
                hp[rb][c] = y;
                __builtin_amdgcn_sched_barrier(0);          // one block at a time: bounded live ranges
            }
    }

    // h^L of the live rows for the orbital head
    if (live && trow) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int c = 0; c < 16; ++c) *(f32x4 *)(a.Hout + row[rb] * a.ldh + 16 * c + 4 * og) = hp[rb][c];
    }
}

bool g_stack_regs = true;

bool stack_regs_supported(int mode, int N, int nu, int TR, int w1, int L, const int *HW, const int *GW)
{
    if (!(mode == GEMM_BF16 || mode == GEMM_BF16W3 || mode == GEMM_BF16W2)) return false;
    if (!g_stack_regs || g_use_stack == 0 || N != 4 || nu != 2 || TR != 16 || w1 != 256 || L < 1 || L > FN_MAX_LAYERS) return false;
    for (int l = 0; l < L; ++l) {
        if (HW[l] % 32 || GW[l] % 32 || HW[l] > 256 || HW[l] + GW[l] > 512) return false;
        if (l >= 1 && HW[l] != 256) return false;
    }
    return true;
}

void launch_stack_regs(int mode, const StackArgs &a, hipStream_t st)
{
    if (a.B <= 0) return;
    const dim3 grid((unsigned)((a.B + 1) / 2)), block(256);
    switch (mode) {
    case GEMM_BF16: hipLaunchKernelGGL(k_stack_regs<1>, grid, block, 0, st, a); break;
    case GEMM_BF16W2: hipLaunchKernelGGL(k_stack_regs<2>, grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL(k_stack_regs<3>, grid, block, 0, st, a); break;
    }
}

}  // namespace fn
