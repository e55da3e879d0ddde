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
constexpr int CPT = 2;                // 16-byte copies per lane per tile (eight waves)

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
// 16 bytes at byte offset voff + soff (soff wave-uniform) of the buffer into
// lds + 16 * lane (lds: the wave's 1 KB block)
__device__ inline void copy16_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, void *lds)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)lds, 16, voff, soff, 0, 0);
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
__global__ __launch_bounds__(512, 1) void k_stack_regs(StackArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char ring[RT * TILE];
    __shared__ __attribute__((aligned(16))) f32x4 pex[2][16][64];       // P of each walker, D layout
    // spin-mean operand slices [step parity][wave][lo, hi] (A phase), and in
    // the same bytes the per-wave epilogue scratch [wave][z_0 -> tanh,
    // Laplacian source term][column] (the epilogue writes the next layer's
    // first slice only after its last read of the scratch)
    __shared__ __attribute__((aligned(16))) float4 slc[2][8][2][64];
    float (*vsc)[2][256] = reinterpret_cast<float (*)[2][256]>(&slc[0][0][0][0]);
    static_assert(sizeof(float) * 8 * 2 * 256 <= sizeof(float4) * 2 * 8 * 2 * 64, "epilogue scratch");

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int t = lane & 15, og = lane >> 4;
    const int wl = wave >> 2, el = wave & 3;          // walker of the workgroup, electron of the walker
    const int sig = el >> 1, half = el & 1;           // spin; which eight column blocks of the spin's P
    const int64_t w = 2 * (int64_t)blockIdx.x + wl;
    const bool live = w < a.B;
    const int64_t wc = live ? w : a.B - 1;           // loads of an absent walker read a valid one
    const int n3 = a.n3, tl = n3 + 1;
    const bool trow = t <= tl;                        // rows past the Laplacian row are padding
    const float ftan = t >= 1 && t <= n3 ? 1.f : 0.f; // tangent rows
    const float flap = t == tl ? 1.f : 0.f;           // Laplacian row
    const float fval = t == 0 ? 1.f : 0.f;            // value row
    const uint32_t vmask = t == 0 ? 0xffffffffu : 0u;
    const int64_t row0 = (wc * 4 + el) * 16;         // this wave's electron
    const int64_t row = row0 + t;
    const int64_t rowp0 = (wc * 4 + 2 * sig) * 16;   // the spin's first electron

    // ---- ring tiles, in consumption order, per layer: for each input step
    //      of h the V_g tiles of both spins and the V_h tile; for each
    //      pair-mean step the V_h tile and then the pair means of every
    //      wave's rows (2 KB per wave, rows chunk-swizzled)
    auto layer_tiles = [&](int l) { return 3 * (a.HW[l] >> 5) + 2 * (a.GW[l] >> 5); };
    int NT = 0;
    for (int l = 0; l < a.L; ++l) NT += layer_tiles(l);
    int il = 0, iu = 0;                              // layer and in-layer index of the next tile to issue
    // lane parts of the copy offsets (the same for every tile): weight tiles
    // row (lane / 4) of a 16-row block, its chunk (lane & 3) swizzled; pair
    // means row (lane / 8) of an 8-row block, chunk (lane & 7) swizzled
    const uint32_t wrow2 = 2u * (uint32_t)(lane >> 2);
    const uint32_t wchunk = 16u * (uint32_t)lds_chunk(lane >> 2, lane & 3);
    const uint32_t glane = (uint32_t)((lane >> 3) * a.ldgi * 4 + 16 * ((lane & 7) ^ ((lane >> 3) & 7)));
    auto issue = [&](int T) {
        const int l = il, u = iu, nH = a.HW[l] >> 5;
        if (++iu == layer_tiles(il)) {
            iu = 0;
            ++il;
        }
        unsigned char *slot = ring + (T % RT) * TILE;
        if (u >= 3 * nH && ((u - 3 * nH) & 1)) {
            // pair means, step g: rows 8 j + lane / 8 of this wave's 16,
            // 16-byte chunk c of the row stored at slot c ^ (row & 7)
            const int g = (u - 3 * nH) >> 1;
            const float *base = a.GI + (int64_t)l * a.gi_stride + row0 * a.ldgi + 32 * g;
            const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(base, (uint32_t)(16 * a.ldgi * 4));
#pragma unroll
            for (int j = 0; j < CPT; ++j)
                copy16_buf(rs, glane, (uint32_t)(8 * j * a.ldgi * 4), slot + wave * 2048 + j * 1024);
            return;
        }
        const uint16_t *W;
        int ld, k0;
        if (u < 3 * nH && u % 3 < 2) {
            W = a.Wg[l];
            ld = 2 * a.HW[l];
            k0 = (u % 3) * a.HW[l] + 32 * (u / 3);
        } else {
            W = a.Wx[l];
            ld = a.HW[l] + a.GW[l];
            k0 = u < 3 * nH ? 32 * (u / 3) : a.HW[l] + 32 * ((u - 3 * nH) >> 1);
        }
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(W + k0, (uint32_t)(256 * ld * 2));
        const uint32_t voff = wrow2 * (uint32_t)ld + wchunk;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int b = CPT * wave + j;
            copy16_buf(rs, voff, (uint32_t)(16 * b * ld * 2), slot + b * 1024);
        }
    };
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
    // (formed again at each use from the lane id: cheaper than keeping it)
    auto afrag_now = [&]() {
        int ln = __lane_id();
        asm volatile("" : "+v"(ln));
        const int tt = ln & 15;
        return tt * 64 + 16 * lds_chunk(tt, ln >> 4);
    };

    f32x4 hp[16];                                     // h of this layer's input (then output), D layout
    f32x4 acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) hp[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float4 own_lo = make_float4(0.f, 0.f, 0.f, 0.f), own_hi = own_lo;   // this step's operand of the wave's electron

    auto feat_operand = [&](int64_t r, int s, float4 &lo, float4 &hi) {
        const float *p = a.H0 + r * a.ldh + 32 * s + 8 * og;
        lo = mask4r(*(const float4 *)p, trow);
        hi = mask4r(*(const float4 *)(p + 4), trow);
    };
    // one input step of h: the spin-mean products of this wave's eight
    // column blocks of P_spin (tile first + spin) and the electron's products
    // over all sixteen blocks (tile first + 2); weight fragments two at a
    // time, the next two requested before a pair's products
    f32x4 pm[8];
    auto step_products = [&](const float4 &plo, const float4 &phi) {
        const float4 mlo = make_float4((own_lo.x + plo.x) * 0.5f, (own_lo.y + plo.y) * 0.5f, (own_lo.z + plo.z) * 0.5f,
                                       (own_lo.w + plo.w) * 0.5f);
        const float4 mhi = make_float4((own_hi.x + phi.x) * 0.5f, (own_hi.y + phi.y) * 0.5f, (own_hi.z + phi.z) * 0.5f,
                                       (own_hi.w + phi.w) * 0.5f);
        bf16x8 ha[NA], hb[NA];
        split_fragment<NA>(mlo, mhi, ha);
        split_fragment<NA>(own_lo, own_hi, hb);
        const int af = afrag_now();
        {
            const unsigned char *tile = ring + ((first + sig) % RT) * TILE + af + 8 * half * 1024;
            bf16x8 wa[2], wn[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) wa[j] = *(const bf16x8 *)(tile + j * 1024);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                asm volatile("" ::: "memory");
                if (g < 3) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wn[j] = *(const bf16x8 *)(tile + (2 * g + 2 + j) * 1024);
                }
#pragma unroll
                for (int p = 0; p < NA; ++p)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        pm[2 * g + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], ha[p], pm[2 * g + j], 0, 0, 0);
                if (g < 3) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
        }
        {
            const unsigned char *tile = ring + ((first + 2) % RT) * TILE + af;
            bf16x8 wa[2], wn[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) wa[j] = *(const bf16x8 *)(tile + j * 1024);
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                asm volatile("" ::: "memory");
                if (g < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wn[j] = *(const bf16x8 *)(tile + (2 * g + 2 + j) * 1024);
                }
#pragma unroll
                for (int p = 0; p < NA; ++p)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[2 * g + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], hb[p], acc[2 * g + j], 0, 0, 0);
                if (g < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
        }
    };

    for (int l = 0; l < a.L; ++l) {
        const int nH = a.HW[l] >> 5, nG = a.GW[l] >> 5;
#pragma unroll
        for (int j = 0; j < 8; ++j) pm[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};

        // ---- input steps of h: P_spin = g_spin V_g^spin with g = (h_e0 + h_e1) / 2
        //      (layer 0: both electrons' features; later layers: this wave's
        //      operand and the partner's slice, stored one step ahead), and
        //      X += h V_h for the wave's electron
        if (l == 0) {
#pragma unroll 1
            for (int s = 0; s < nH; ++s) {
                step_sync(first + 3);
                float4 plo, phi;
                feat_operand(row, s, own_lo, own_hi);
                feat_operand(((wc * 4) + (el ^ 1)) * 16 + t, s, plo, phi);
                step_products(plo, phi);
                first += 3;
            }
        } else {
            // (unrolled: static register indices for the next step's operand)
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (s >= nH) break;
                step_sync(first + 3);
                const float4 plo = slc[s & 1][wave ^ 1][0][lane], phi = slc[s & 1][wave ^ 1][1][lane];
                float4 nlo = own_lo, nhi = own_hi;
                if (s + 1 < nH) {
                    d_to_b(hp[2 * s + 2], hp[2 * s + 3], nlo, nhi);
                    slc[(s + 1) & 1][wave][0][lane] = nlo;
                    slc[(s + 1) & 1][wave][1][lane] = nhi;
                }
                step_products(plo, phi);
                own_lo = nlo;
                own_hi = nhi;
                first += 3;
            }
        }
        // P = P_up + P_dn: the spin-up waves store their blocks, the spin-down
        // waves add theirs after the barrier (complete before the barrier of
        // the first pair-mean step)
        if (sig == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) pex[wl][8 * half + j][lane] = pm[j];
        }
        ring_barrier();
        if (sig == 1) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                f32x4 v = pex[wl][8 * half + j][lane];
                v += pm[j];
                pex[wl][8 * half + j][lane] = v;
            }
        }

        // ---- pair-mean steps: the V_h tile, then this wave's pair-mean rows
#pragma unroll 1
        for (int g = 0; g < nG; ++g) {
            step_sync(first + 2);
            const unsigned char *gt = ring + ((first + 1) % RT) * TILE + wave * 2048 + t * 128;
            const float4 lo = mask4r(*(const float4 *)(gt + 16 * ((2 * og) ^ (t & 7))), trow);
            const float4 hi = mask4r(*(const float4 *)(gt + 16 * ((2 * og + 1) ^ (t & 7))), trow);
            bf16x8 hb[NA];
            split_fragment<NA>(lo, hi, hb);
            const unsigned char *tile = ring + (first % RT) * TILE + afrag_now();
            bf16x8 wa[2], wn[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) wa[j] = *(const bf16x8 *)(tile + j * 1024);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                asm volatile("" ::: "memory");
                if (q < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wn[j] = *(const bf16x8 *)(tile + (2 * q + 2 + j) * 1024);
                }
#pragma unroll
                for (int p = 0; p < NA; ++p)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[2 * q + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], hb[p], acc[2 * q + j], 0, 0, 0);
                if (q < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
            first += 2;
        }

        // ---- epilogue, branch-free: row roles as multipliers and selects;
        //      padding rows come out zero (their z is exactly zero).
        //      Pass 1: z = (X + P) + b; per column the value row z_0 and the
        //      sum over the tangent rows of z_c^2 to the wave's scratch.
        //      Pass 2 (four columns per lane): y_0 = tanh(z_0) and the
        //      Laplacian row's source term 2 y_0 (1 - y_0^2) sum_c z_c^2.
        //      Pass 3: every row of the new h, plus the residual.
        float *z0s = vsc[wave][0], *lts = vsc[wave][1];
        const float *bl = a.bias[l];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            asm volatile("" ::: "memory");
            const f32x4 P = pex[wl][c][lane];
            const float4 b4 = *(const float4 *)(bl + 16 * c + 4 * og);
            const f32x4 bv = f32x4{b4.x * fval, b4.y * fval, b4.z * fval, b4.w * fval};
            const f32x4 z = (acc[c] + P) + bv;                // (X + P) + b on the value row
            acc[c] = z;
            f32x4 sq;
#pragma unroll
            for (int e = 0; e < 4; ++e) sq[e] = sum16((z[e] * z[e]) * ftan);
            if (t == 0) *(f32x4 *)(z0s + 16 * c + 4 * og) = z;
            if (t == tl) *(f32x4 *)(lts + 16 * c + 4 * og) = sq;
            __builtin_amdgcn_sched_barrier(0);
        }
        {
            const float4 u = *(const float4 *)(z0s + 4 * lane);
            const float4 q = *(const float4 *)(lts + 4 * lane);
            const float4 y = make_float4(tanhf(u.x), tanhf(u.y), tanhf(u.z), tanhf(u.w));
            const float4 d = make_float4(1.f - y.x * y.x, 1.f - y.y * y.y, 1.f - y.z * y.z, 1.f - y.w * y.w);
            *(float4 *)(z0s + 4 * lane) = y;
            *(float4 *)(lts + 4 * lane) = make_float4(2.f * y.x * d.x * q.x, 2.f * y.y * d.y * q.y, 2.f * y.z * d.z * q.z,
                                                      2.f * y.w * d.w * q.w);
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            asm volatile("" ::: "memory");                     // this block's reads stay in its iteration
            const float4 y4 = *(const float4 *)(z0s + 16 * c + 4 * og);
            const float4 l4 = *(const float4 *)(lts + 16 * c + 4 * og);
            const float y0[4] = {y4.x, y4.y, y4.z, y4.w};
            const float dd[4] = {1.f - y4.x * y4.x, 1.f - y4.y * y4.y, 1.f - y4.z * y4.z, 1.f - y4.w * y4.w};
            const float lt[4] = {l4.x, l4.y, l4.z, l4.w};
            const f32x4 z = acc[c];
            f32x4 y;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = dd[e] * z[e] - flap * lt[e];         // tangent rows; Laplacian row with its source
                // value row: y_0 (a bit select, so no branch), plus the residual (zero before layer 1)
                y[e] = __uint_as_float((__float_as_uint(y0[e]) & vmask) | (__float_as_uint(v) & ~vmask)) + hp[c][e];
            }
            hp[c] = y;
            asm volatile("" : "+a"(hp[c]));                    // h lives in the accumulator registers
            __builtin_amdgcn_sched_barrier(0);
        }
        // the next layer's first operand of this wave's electron, and its slice
        // for the partner
        if (l + 1 < a.L) {
            d_to_b(hp[0], hp[1], own_lo, own_hi);
            slc[0][wave][0][lane] = own_lo;
            slc[0][wave][1][lane] = own_hi;
        }
    }

    // h^L of the live rows for the orbital head
    if (live && trow) {
#pragma unroll
        for (int c = 0; c < 16; ++c) *(f32x4 *)(a.Hout + row * a.ldh + 16 * c + 4 * og) = hp[c];
    }
}

bool g_stack_regs = true;

bool stack_regs_supported(int mode, int N, int nu, int TR, int w1, int L, const int *HW, const int *GW)
{
    if (!(mode == GEMM_BF16 || mode == GEMM_BF16W3 || mode == GEMM_BF16W2)) return false;
    if (!g_stack_regs || g_use_stack == 0 || N != 4 || nu != 2 || TR != 16 || w1 != 256 || L < 1 || L > FN_MAX_LAYERS) return false;
    for (int l = 0; l < L; ++l) {
        // (at least one input step and one pair-mean step: their barriers
        // order the exchange of P and of the operand slices)
        if (HW[l] % 32 || GW[l] % 32 || HW[l] < 32 || GW[l] < 32 || HW[l] > 256 || HW[l] + GW[l] > 512) return false;
        if (l >= 1 && HW[l] != 256) return false;
    }
    return true;
}

void launch_stack_regs(int mode, const StackArgs &a, hipStream_t st)
{
    if (a.B <= 0) return;
    const dim3 grid((unsigned)((a.B + 1) / 2)), block(512);
    switch (mode) {
    case GEMM_BF16: hipLaunchKernelGGL(k_stack_regs<1>, grid, block, 0, st, a); break;
    case GEMM_BF16W2: hipLaunchKernelGGL(k_stack_regs<2>, grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL(k_stack_regs<3>, grid, block, 0, st, a); break;
    }
}

}  // namespace fn
