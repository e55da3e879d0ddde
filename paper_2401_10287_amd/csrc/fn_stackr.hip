// fn_stackr.hip -- every one-electron stream layer of a forward-Laplacian
// pass (FermiNet Model section of the paper) in one kernel with the
// activations held in registers, for walkers of four electrons, two of each
// spin (16 rows per electron: value, 12 tangents, Laplacian, padding),
// w1 = 256, in the modes whose layer weights are one BF16 part (activations
// split into NA exact-or-rounded BF16 parts).
//
// Workgroup: eight waves and two walkers.  Wave q owns electron q & 3 of
// walker q >> 2 (electrons stored spin-up first, so waves q and q ^ 1 hold
// the two electrons of one spin), all 256 output columns of its 16 rows.
// Every product runs transposed,
//   D^T = W^T X^T,
// so the weight fragments (rows = output columns) are the matrix
// instruction's A operand, read from an LDS ring that the eight waves share,
// and the activations are the B operand, taken from the wave's own
// registers.  Accumulator ("D") layout: lane (t = lane % 16, og = lane / 16)
// of block c holds output columns 16 c + 4 og + e, e = 0..3, of row t.  The
// B operand of reduction step s (input columns 32 s + 8 kg .. + 7 of row t
// in lane (t, kg)) is formed from blocks 2 s and 2 s + 1 of the previous
// layer's output by one 32-lane and one 16-lane swap per element.
//
// Per layer l:
//   input steps s of h (one barrier each): P_spin += g_spin V_g^spin for
//            eight of the sixteen column blocks (g = mean of the wave's and
//            its partner's operand, the partner's through LDS), and
//            X += h V_h for the wave's electron;
//   exchange: the spin-up waves store P_up, the spin-down waves add P_dn
//            (P, the same for all four electrons of the walker);
//   pair-mean steps: X += [g_i_up | g_i_dn] V_h (the pair means come
//            through the ring as well, each wave its own rows, with the
//            layer's bias in their padding rows);
//   epilogue in registers: z = X + P, value y = tanh(z_0 + b), tangents
//            (1 - y^2) z_c, Laplacian (1 - y^2) z_L - 2 y (1 - y^2) sum_c
//            z_c^2 (the sum over the tangent rows by a transpose through
//            the wave's LDS scratch), residual.
// Weights stream through the ring as 16 KB tiles (256 output rows x 32
// reduction columns) by direct global-to-LDS copies a step ahead, issued
// between the products; each step waits only for its own tiles.  Only the
// features, the pair means and h^L touch HBM.
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

namespace {

constexpr int RT = 6;                 // ring tiles of 16 KB
constexpr int TILE = 16384;
constexpr int CPT = 2;                // 16-byte copies per lane per tile (eight waves)
constexpr int N3 = 12;                // tangent rows: three coordinates of four electrons

// until at most CPT * n vector-memory operations of this wave are
// outstanding (n tiles still in flight).  Loads complete in order, so this
// lands every older tile; a pair-mean tile takes one copy more than CPT (its
// padding rows bring the bias), which only makes the wait stricter
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

__device__ inline float4 mask4r(float4 x, bool keep) { return keep ? x : make_float4(0.f, 0.f, 0.f, 0.f); }

}  // namespace

template <int NA>
__global__ __launch_bounds__(512, 1) void k_stack_regs(StackArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char ring[RT * TILE];
    __shared__ __attribute__((aligned(16))) f32x4 pex[2][16][64];       // P of each walker, D layout
    // operand slices for the partner wave [step parity][wave][lo, hi]; the
    // two slices of a wave are also its epilogue scratch
    __shared__ __attribute__((aligned(16))) float4 slc[2][8][2][64];

    __builtin_amdgcn_s_setprio(1);                    // (0 while issuing copies)
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int t = lane & 15, og = lane >> 4;
    const int wl = wave >> 2, el = wave & 3;          // walker of the workgroup, electron of the walker
    const int sig = el >> 1, half = el & 1;           // spin; which eight column blocks of the spin's P
    const int64_t w = 2 * (int64_t)blockIdx.x + wl;
    const bool live = w < a.B;
    const int64_t wc = live ? w : a.B - 1;           // loads of an absent walker read a valid one
    const bool trow = t <= N3 + 1;                    // rows past the Laplacian row are padding
    const int64_t row0 = (wc * 4 + el) * 16;         // this wave's electron
    const int64_t row = row0 + t;

    // ---- ring tiles, in consumption order, per layer: for each input step
    //      of h the V_g tiles of both spins and the V_h tile; for each
    //      pair-mean step the V_h tile and then the pair means of every
    //      wave's rows (2 KB per wave, rows chunk-swizzled)
    const bool head = a.WH[0] != nullptr;
    int NT = 0;
    for (int l = 0; l < a.L; ++l) NT += 3 * (a.HW[l] >> 5) + 2 * (a.GW[l] >> 5);
    // lane parts of the copy offsets (the same for every tile): weight tiles
    // row (lane / 4) of a 16-row block, its chunk (lane & 3) swizzled; pair
    // means row (lane / 8) of an 8-row block, chunk (lane & 7) swizzled
    const uint32_t wrow2 = 2u * (uint32_t)(lane >> 2);
    const uint32_t wchunk = 16u * (uint32_t)lds_chunk(lane >> 2, lane & 3);
    const uint32_t glane = (uint32_t)((lane >> 3) * a.ldgi * 4 + 16 * ((lane & 7) ^ ((lane >> 3) & 7)));
    // position of the next tile to issue: layer il, phase iph (0: input
    // steps of h, 1: pair-mean steps), step is, tile ir of the step; the
    // layer's weights and widths are read once per layer
    int il = 0, iph = 0, is = 0, ir = 0, islot = 0;
    const uint16_t *iWg = a.Wg[0], *iWx = a.Wx[0];
    int iHW = a.HW[0], iGW = a.GW[0];
    const float *igi = a.GI + row0 * a.ldgi, *ibias = a.bias[0];
    // the copies of the next tile, then the position moves on
    auto issue = [&]() {
        unsigned char *slot = ring + islot * TILE;
        if (iph == 1 && ir == 1) {
            // pair means, step is: rows 8 j + lane / 8 of this wave's 16,
            // 16-byte chunk c of the row stored at slot c ^ (row & 7).  Rows
            // 14 and 15 are padding: their lanes bring 64 bias values of the
            // layer instead (columns 64 (wave & 3) .. + 63, in order), which
            // the epilogue reads while the slot stays untouched
            const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(igi + 32 * is, (uint32_t)(16 * a.ldgi * 4));
            copy16_buf(rs, glane, 0u, slot + wave * 2048);
            if (lane < 48)
                copy16_buf(rs, glane, (uint32_t)(8 * a.ldgi * 4), slot + wave * 2048 + 1024);
            else
                copy16_buf(buffer_rsrc(ibias, 256 * 4), (uint32_t)(16 * (lane - 48)), (uint32_t)(256 * (wave & 3)),
                           slot + wave * 2048 + 1024);
        } else {
            const uint16_t *W;
            int ld;
            if (iph == 0 && ir < 2) {
                W = iWg + ir * iHW + 32 * is;
                ld = 2 * iHW;
            } else {
                W = iWx + (iph ? iHW : 0) + 32 * is;
                ld = iHW + iGW;
            }
            const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(W, (uint32_t)(256 * ld * 2));
            const uint32_t voff = wrow2 * (uint32_t)ld + wchunk;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int b = CPT * wave + j;
                copy16_buf(rs, voff, (uint32_t)(16 * b * ld * 2), slot + b * 1024);
            }
        }
        if (++islot == RT) islot = 0;
        if (++ir < 3 - iph) return;
        ir = 0;
        if (++is < (iph ? iGW : iHW) >> 5) return;
        is = 0;
        if (iph == 0) {
            iph = 1;
            return;
        }
        iph = 0;
        if (++il < a.L) {
            iWg = a.Wg[il];
            iWx = a.Wx[il];
            iHW = a.HW[il];
            iGW = a.GW[il];
            igi += a.gi_stride;
            ibias = a.bias[il];
        }
    };
    int issued = 0, first = 0;
    // every lane has landed the tiles before `need`, then the workgroup
    // agrees; tiles that no step before `first` still reads are refilled
    // (the refills go out between the step's matrix instructions, a tile at
    // a time, so that no wave waits for a queue of copies before its first
    // products; any left over go out at the next step's start)
    auto step_sync = [&](int need) {
        wait_tiles(issued - need);
        ring_barrier();
        for (; issued < NT && issued < first - 3 + RT; ++issued) issue();
    };
    // refill position p of a step (p static): a whole tile at positions 0,
    // 4 and 8 (each burst of copies drains before the next one queues up;
    // closer positions, or the two walkers' waves at alternating positions,
    // measured slower).  The wave drops to the lower priority while it
    // issues its copies, so that a wave with products to issue goes first
    auto refill_at = [&](int p) {
        if ((p == 0 || p == 4 || p == 8) && issued < NT && issued < first + RT) {
            __builtin_amdgcn_s_setprio(0);
            issue();
            __builtin_amdgcn_s_setprio(1);
            ++issued;
        }
    };
    for (; issued < NT && issued < RT; ++issued) issue();
    // ring slot of tile first + k (k < RT)
    int fslot = 0;
    auto slot_of = [&](int k) { return fslot + k < RT ? fslot + k : fslot + k - RT; };
    auto advance = [&](int k) {
        first += k;
        fslot = slot_of(k);
    };

    // A fragment of output block c in a ring tile: row 16 c + t, chunk og
    // (formed again at each use from the lane id: cheaper than keeping it)
    auto afrag_now = [&]() {
        int ln = __lane_id();
        asm volatile("" : "+v"(ln));
        const int tt = ln & 15;
        return tt * 64 + 16 * lds_chunk(tt, ln >> 4);
    };

    // this lane's 16-byte slot in a 1 KB row of LDS, formed at each use (the
    // compiler would otherwise keep one such offset per array and wave)
    auto lane_slot = [&](void *base) {
        int ln = __lane_id();
        asm volatile("" : "+v"(ln));
        return reinterpret_cast<f32x4 *>(reinterpret_cast<unsigned char *>(base) + 16 * ln);
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
    // one input step of h: the electron's products over all sixteen blocks
    // (tile first + 2) and the spin-mean products of this wave's eight
    // column blocks of P_spin (tile first + spin); weight fragments two at a
    // time, the next two requested before a pair's products; refills after
    // product groups 0, 4 and 8 of the step's twelve
    f32x4 pm[8];
    auto step_products = [&](const float4 &plo, const float4 &phi) {
        bf16x8 ha[NA], hb[NA];
        auto mean_operand = [&]() {
            const float4 mlo = make_float4((own_lo.x + plo.x) * 0.5f, (own_lo.y + plo.y) * 0.5f,
                                           (own_lo.z + plo.z) * 0.5f, (own_lo.w + plo.w) * 0.5f);
            const float4 mhi = make_float4((own_hi.x + phi.x) * 0.5f, (own_hi.y + phi.y) * 0.5f,
                                           (own_hi.z + phi.z) * 0.5f, (own_hi.w + phi.w) * 0.5f);
            split_fragment<NA>(mlo, mhi, ha);
        };
        // with several activation parts the electron's products go first and
        // the spin-mean operand is formed and split while the first of them
        // run; with one part (short product groups) the spin-mean products
        // go first
        constexpr bool own_first = NA > 1;
        split_fragment<NA>(own_lo, own_hi, hb);
        if (!own_first) mean_operand();
        const int af = afrag_now();
        auto own_products = [&](int p0) {
            const unsigned char *tile = ring + slot_of(2) * TILE + af;
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
                if (own_first && g == 0) mean_operand();
                refill_at(p0 + g);
                if (g < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
        };
        auto mean_products = [&](int p0) {
            const unsigned char *tile = ring + slot_of(sig) * TILE + af + 8 * half * 1024;
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
                refill_at(p0 + g);
                if (g < 3) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
        };
        if (own_first) {
            own_products(0);
            mean_products(8);
        } else {
            mean_products(0);
            own_products(4);
        }
        // the electron's sums live in the accumulator registers between steps
#pragma unroll
        for (int c = 0; c < 16; ++c) asm volatile("" : "+a"(acc[c]));
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
                advance(3);
            }
        } else {
            // (unrolled: static register indices for the next step's operand)
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (s >= nH) break;
                step_sync(first + 3);
                const f32x4 *const ps = lane_slot(&slc[s & 1][wave ^ 1][0][0]);
                const float4 plo = *(const float4 *)ps, phi = *(const float4 *)(ps + 64);
                step_products(plo, phi);
                // the next step's operand, and its slice for the partner
                // (formed after the products: not live through them)
                if (s + 1 < nH) {
                    d_to_b(hp[2 * s + 2], hp[2 * s + 3], own_lo, own_hi);
                    f32x4 *const ns = lane_slot(&slc[(s + 1) & 1][wave][0][0]);
                    *(float4 *)ns = own_lo;
                    *(float4 *)(ns + 64) = own_hi;
                }
                advance(3);
            }
        }
        // P = P_up + P_dn: the spin-up waves store their blocks, the spin-down
        // waves add theirs after the barrier (complete before the barrier of
        // the first pair-mean step)
        if (sig == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) lane_slot(&pex[wl][8 * half][0])[64 * j] = pm[j];
        }
        ring_barrier();
        if (sig == 1) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                f32x4 *const pp = lane_slot(&pex[wl][8 * half][0]) + 64 * j;
                *pp = *pp + pm[j];
            }
        }

        // ---- pair-mean steps: the V_h tile, then this wave's pair-mean rows
        int gi_slot = 0;
#pragma unroll 1
        for (int g = 0; g < nG; ++g) {
            step_sync(first + 2);
            gi_slot = slot_of(1);
            // (lane offsets formed here from the lane id, not kept across the loop)
            int ln = __lane_id();
            asm volatile("" : "+v"(ln));
            const int lt = ln & 15, lg = ln >> 4;
            const unsigned char *gt = ring + gi_slot * TILE + wave * 2048 + lt * 128;
            const float4 lo = mask4r(*(const float4 *)(gt + 16 * ((2 * lg) ^ (lt & 7))), trow);
            const float4 hi = mask4r(*(const float4 *)(gt + 16 * ((2 * lg + 1) ^ (lt & 7))), trow);
            bf16x8 hb[NA];
            split_fragment<NA>(lo, hi, hb);
            const unsigned char *tile = ring + fslot * TILE + afrag_now();
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
                refill_at(q);
                if (q < 7) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) wa[j] = wn[j];
                }
            }
            advance(2);
        }

        // ---- epilogue.  Scratch of this wave: its two operand slices
        //      (sA, sB: 2 KB each, free until it writes the next layer's
        //      first slice at the end).
        //      Pass 1, four chunks of 64 columns: z = X + P; rows 0-12
        //      staged (rows 0-6 in sA, 7-12 in sB, 68 floats apart), then
        //      lane j reads column j: the value row z_0 and the sum over the
        //      tangent rows of z_c^2.
        //      Pass 2, the four columns 64 q + lane: y_0 = tanh(z_0 + b),
        //      d = 1 - y_0^2 and the Laplacian source -2 y_0 d sum_c z_c^2,
        //      into per-column tables.
        //      Pass 3: every row as A z + C with (A, C) by row role: value
        //      (0, y_0), tangent and padding (d, 0), Laplacian (d, source);
        //      then the residual.
        if (head && l + 1 == a.L) {
            // the head weights of both spins into the next two ring slots
            // (their tiles were read before the pair-mean step: free now);
            // they land while the epilogue runs.  Spin sp's tile: 1 KB block
            // b = 2 s + c holds output rows 16 c .. + 15, reduction columns
            // 32 s .. + 31 (s = wave)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp) {
                const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(a.WH[sp], (uint32_t)(32 * a.ldwh * 2));
                const uint32_t voff = wrow2 * (uint32_t)a.ldwh + wchunk;
                unsigned char *slot = ring + slot_of(sp) * TILE;
#pragma unroll
                for (int j = 0; j < CPT; ++j)
                    copy16_buf(rs, voff, (uint32_t)((16 * j * a.ldwh + 32 * wave) * 2), slot + (CPT * wave + j) * 1024);
            }
        }
        float *const sA = &slc[0][wave][0][0].x, *const sB = &slc[1][wave][0][0].x;
        // (lane-dependent offsets formed here from the lane id, not kept
        // across the layer loop)
        int ln = __lane_id();
        asm volatile("" : "+v"(ln));
        const int lt = ln & 15, lg = ln >> 4;
        float z0[4], sq[4];
        {
            constexpr int RS = 68;                               // staged row stride (floats)
            constexpr int SB = (int)(sizeof(slc[0]) / sizeof(float));   // sB - sA
            float *const srow = (lt < 7 ? sA + RS * lt : sB + RS * (lt - 7)) + 4 * lg;
            const f32x4 *const pl = lane_slot(&pex[wl][0][0]);
            f32x4 pn = pl[0];                                   // P of the next block, read one ahead
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const int c = 4 * q + cc;
                    const f32x4 P = pn;
                    if (c < 15) pn = pl[64 * (c + 1)];
                    const f32x4 z = acc[c] + P;
                    acc[c] = z;
                    if (lt <= N3) *(f32x4 *)(srow + 16 * cc) = z;
                    __builtin_amdgcn_sched_barrier(0);
                }
                asm volatile("" ::: "memory");
                const float *const col = sA + ln;
                z0[q] = col[0];
                float v = 0.f;
#pragma unroll
                for (int r = 1; r <= N3; ++r) {
                    const float x = col[r < 7 ? RS * r : SB + RS * (r - 7)];
                    v = r == 1 ? x * x : fmaf(x, x, v);
                }
                sq[q] = v;
                asm volatile("" ::: "memory");
            }
        }
        float *const y0T = sA, *const ddT = sA + 256, *const srcT = sB, *const zeroT = sB + 256;
        // the bias, from the padding rows of the last pair-mean tile
        const float *const bsl = reinterpret_cast<const float *>(ring + gi_slot * TILE + 1792);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float y = tanhf(z0[q] + bsl[512 * q + ln]);
            const float d = 1.f - y * y;
            y0T[64 * q + ln] = y;
            ddT[64 * q + ln] = d;
            srcT[64 * q + ln] = -(2.f * y * d * sq[q]);
        }
        *(float4 *)(zeroT + 4 * ln) = make_float4(0.f, 0.f, 0.f, 0.f);
        asm volatile("" ::: "memory");
        {
            const float *const tA = (lt == 0 ? zeroT : ddT) + 4 * lg;
            const float *const tC = (lt == 0 ? y0T : (lt == N3 + 1 ? srcT : zeroT)) + 4 * lg;
            float4 An = *(const float4 *)tA, Cn = *(const float4 *)tC;   // read one block ahead
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const float4 A4 = An, C4 = Cn;
                if (c < 15) {
                    An = *(const float4 *)(tA + 16 * (c + 1));
                    Cn = *(const float4 *)(tC + 16 * (c + 1));
                }
                const f32x4 z = acc[c];
                f32x4 y;
                y[0] = fmaf(A4.x, z[0], C4.x);
                y[1] = fmaf(A4.y, z[1], C4.y);
                y[2] = fmaf(A4.z, z[2], C4.z);
                y[3] = fmaf(A4.w, z[3], C4.w);
                hp[c] = y + hp[c];                               // residual (zero before layer 1)
                asm volatile("" : "+a"(hp[c]));                  // h lives in the accumulator registers
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        asm volatile("" ::: "memory");
        // the next layer's first operand of this wave's electron, and its slice
        // for the partner
        // (also after the last layer: unconditional, so that the previous
        // operand is dead through the epilogue)
        d_to_b(hp[0], hp[1], own_lo, own_hi);
        {
            f32x4 *const ns = lane_slot(&slc[0][wave][0][0]);
            *(float4 *)ns = own_lo;
            *(float4 *)(ns + 64) = own_hi;
        }
    }

    if (!head) {
        // h^L of the live rows for the orbital head
        if (live && trow) {
#pragma unroll
            for (int c = 0; c < 16; ++c) *(f32x4 *)(a.Hout + row * a.ldh + 16 * c + 4 * og) = hp[c];
        }
        return;
    }
    // the orbital head (FermiNet Model section): O = h^L w for the wave's
    // electron, K n = 32 outputs of its spin, from h^L in registers and the
    // spin's head weights (tile first + spin), in the layers' product form
    wait_tiles(0);
    ring_barrier();
    f32x4 ho[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    {
        const unsigned char *tile = ring + slot_of(sig) * TILE + afrag_now();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            float4 lo, hi;
            d_to_b(hp[2 * s], hp[2 * s + 1], lo, hi);
            bf16x8 hb[NA];
            split_fragment<NA>(lo, hi, hb);
            const bf16x8 w0 = *(const bf16x8 *)(tile + (2 * s) * 1024);
            const bf16x8 w1 = *(const bf16x8 *)(tile + (2 * s + 1) * 1024);
#pragma unroll
            for (int p = 0; p < NA; ++p) {
                ho[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, hb[p], ho[0], 0, 0, 0);
                ho[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, hb[p], ho[1], 0, 0, 0);
            }
        }
    }
    if (live && trow) {
        float *o = a.O[sig] + ((wc * 2 + half) * 16 + t) * a.ldo[sig] + 4 * og;
#pragma unroll
        for (int c = 0; c < 2; ++c) *(f32x4 *)(o + 16 * c) = ho[c];
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
