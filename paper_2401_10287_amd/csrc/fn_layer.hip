// fn_layer.hip -- one one-electron stream layer (FermiNet Model section of the
// paper) as a single kernel:
//   z = [h_i | g_i_up | g_i_dn] V_h + P_walker + b (value row),
//   h^{l+1} = tanh(z) (+ h^l)
// in forward-Laplacian form: value row y = tanh(z_0), tangent rows
// (1 - y^2) dz_c, Laplacian row (1 - y^2) lap z - 2 y (1 - y^2) sum_c dz_c^2.
//
// Tiles: 128 rows x 128 columns per 256-thread workgroup, the two column
// halves of a row block on one XCD back to back; each wave64 owns a
// 64 x 64 quarter as 4 x 4 blocks of 16 x 16 MFMA accumulators.  Operand
// tiles of 32 reduction steps are staged through LDS, the next tile's global
// loads issued before the current tile's matrix instructions; split-BF16
// operand fragments are loaded once and reused by every product of parts.
// In the split-BF16 modes the copies go straight from global memory into a
// two-stage LDS ring (FP32 activations, pre-split weights), and each wave
// splits its activation fragments as it reads them; otherwise the loads are
// staged through registers and split once as they are stored.
// Each electron owns TP rows (TP = 1 value only, or 16 / 32 / 64), so an
// electron never straddles a tile.  The epilogue parks the pre-activations
// in LDS (over the operand stage) and finishes each (electron, column) pair
// in one thread: value row, tangent rows and the Laplacian row with its
// source sum_c dz_c^2.  Output widths up to 256 columns.
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {


namespace {

constexpr int LBM = 128, LBK = 32;

// bitwise select (m all ones or zero) without a branch
__device__ inline float4 mask4(float4 x, uint32_t m)
{
    return make_float4(__uint_as_float(__float_as_uint(x.x) & m), __uint_as_float(__float_as_uint(x.y) & m),
                       __uint_as_float(__float_as_uint(x.z) & m), __uint_as_float(__float_as_uint(x.w) & m));
}
constexpr int LDH = LBK;          // BF16 tile rows, chunk-swizzled (lds_chunk)
constexpr int LDF = LBK + 4;

}  // namespace

// LBN = 128: 2 x 2 waves of 64 x 64; LBN = 32 (value rows only, for grids
// that would leave CUs idle): 4 x 1 waves of 32 x 32.  LIVE: 16-row blocks
// of an electron that hold live rows (value .. Laplacian); with TP = 64 a
// wave's four row blocks are one electron's, and blocks past LIVE (padding
// only, zero in and out) take no matrix instructions.
// DMA: split-BF16 modes with 128-column tiles only.  Activation tiles (FP32)
// and weight tiles (BF16 parts) go from global memory straight into one of
// two LDS stages; each wave splits its own activation fragments when it
// reads them.  One barrier per reduction step, no register staging.
template <int MODE, int TP, int LBN, int LIVE, bool DMA>
__global__ __launch_bounds__(256) void k_stream_layer(LayerArgs a)
{
    static_assert(LBN == 128 || (LBN == 32 && TP == 1), "column tile");
    static_assert(!DMA || (LBN == 128 && MODE != GEMM_F32), "staged copies");
    static_assert(LIVE == (TP + 15) / 16 || (TP == 64 && LBN == 128 && LIVE == 3), "live row blocks");
    constexpr int WI = LBN == 128 ? 4 : 2, WJ = LBN == 128 ? 4 : 2;   // 16 x 16 blocks per wave
    constexpr bool F32 = MODE == GEMM_F32;
    constexpr int NA = act_parts(MODE), NW = weight_parts(MODE);   // BF16 parts of activations / weights
    // one operand stage (A then B); the epilogue reuses it for a 128 x 64 tile
    constexpr int ASZ = F32 ? LBM * LDF * 4 : NA * LBM * LDH * 2;
    constexpr int BSZ = F32 ? LBN * LDF * 4 : NW * LBN * LDH * 2;
    constexpr int XS = LBN + 4;                      // float4-aligned rows of the pre-activation tile
    constexpr int XSZ = LBM * XS * 4;
    constexpr int ESZ = XSZ + 256 * 16;              // tile + partial Laplacian sources
    constexpr int AST = LBM * LBK * 4;               // DMA stage: FP32 activations, then NW weight parts
    constexpr int STG = AST + NW * LBN * LBK * 2;
    constexpr int MSZ = DMA ? 2 * STG : ASZ + BSZ;
    constexpr int SMEM = MSZ > ESZ ? MSZ : ESZ;
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];

    int64_t rb;
    int cb;
    if constexpr (LBN == 128) {
        xcd_tile(blockIdx.x, (a.W1p + LBN - 1) / LBN, rb, cb);
    } else {
        const int64_t nrb = (a.rows + LBM - 1) / LBM;     // row blocks, then column blocks
        rb = blockIdx.x % nrb;
        cb = (int)(blockIdx.x / nrb);
    }
    const int64_t m0 = rb * LBM;
    const int n0 = cb * LBN;
    if (m0 >= a.rows || n0 >= a.W1p) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = LBN == 128 ? wave >> 1 : wave, wn = LBN == 128 ? wave & 1 : 0;
    const int ktiles = (a.K1 + a.K2) / LBK;
    const float *__restrict__ A1 = a.A1;
    const float *__restrict__ A2 = a.A2;

    // per-thread element offsets of the float4s this thread loads: activation
    // rows (clamped to a valid row; out-of-range rows load and are zeroed) for
    // either operand part, and weight rows
    // Padding rows (past an electron's Laplacian row) are not fetched: they
    // take the address of that Laplacian row, which another lane fetches
    // anyway, and are zeroed like out-of-range rows.
    int64_t offa1[4], offa2[4];
    uint32_t aval[4];                                // all ones for a live in-range row, else 0
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int f = tid + 256 * v;
        const int64_t row = m0 + (f >> 3);
        const int lr = TP > 1 ? (f >> 3) % TP : 0;    // row within the electron (tiles start at electrons)
        const bool pad = TP > 1 && lr > a.n3 + 1;
        aval[v] = row < a.rows && !pad ? 0xffffffffu : 0u;
        int64_t rr = m0;
        if (row < a.rows) rr = pad ? row - (lr - (a.n3 + 1)) : row;
        offa1[v] = rr * a.lda1 + 4 * (f & 7);
        offa2[v] = rr * a.lda2 + 4 * (f & 7);
    }
    // weight vectors per thread (per part): FP32 LBN x 8 float4, BF16 LBN x 4 uint4
    constexpr int NBT = F32 ? LBN * 8 : LBN * 4;
    constexpr int NBV = (NBT + 255) / 256;
    int64_t offw[NBV];
    uint32_t wval[NBV];
#pragma unroll
    for (int v = 0; v < NBV; ++v) {
        const int f = tid + 256 * v;
        const int o = F32 ? n0 + (f >> 3) : n0 + (f >> 2);
        const bool ok = f < NBT && o < a.nout;
        wval[v] = ok ? 0xffffffffu : 0u;
        offw[v] = (int64_t)(ok ? o : n0) * a.ldw + (F32 ? 4 * (f & 7) : 8 * (f & 3));
    }
    float4 ra[4];
    uint4 rwh[F32 ? 1 : NBV * NW];
    float4 rwf[F32 ? NBV : 1];

    auto load_tile = [&](int kt) {
        const int kb = kt * LBK;
        // a reduction tile lies wholly in one operand part (K1 is a multiple of LBK)
        if (kb < a.K1) {
            const float *base = A1 + kb;
#pragma unroll
            for (int v = 0; v < 4; ++v) ra[v] = *(const float4 *)(base + offa1[v]);
        } else {
            const float *base = A2 + (kb - a.K1);
#pragma unroll
            for (int v = 0; v < 4; ++v) ra[v] = *(const float4 *)(base + offa2[v]);
        }
        // loads are unconditional (clamped rows); out-of-range rows are
        // zeroed when stored, so no load sits behind a branch
        if constexpr (F32) {
            const float *W = (const float *)a.W + kb;
#pragma unroll
            for (int v = 0; v < NBV; ++v) rwf[v] = *(const float4 *)(W + offw[v]);
        } else {
            const uint16_t *W = (const uint16_t *)a.W + kb;
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int v = 0; v < NBV; ++v) rwh[q * NBV + v] = *(const uint4 *)(W + (int64_t)q * a.wpart + offw[v]);
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int f = tid + 256 * v;
            const int r = f >> 3, k = 4 * (f & 7);
            const float4 x = mask4(ra[v], aval[v]);
            if constexpr (F32) {
                *(float4 *)((float *)smem + r * LDF + k) = x;
            } else {
                uint32_t h01[NA], h23[NA];
                split_bf16_pair<NA>(x.x, x.y, h01);
                split_bf16_pair<NA>(x.z, x.w, h23);
#pragma unroll
                for (int q = 0; q < NA; ++q)
                    *(uint2 *)((uint16_t *)smem + q * LBM * LDH + r * LDH + 8 * lds_chunk(r, k >> 3) + (k & 7)) =
                        make_uint2(h01[q], h23[q]);
            }
        }
        if constexpr (F32) {
            float *sB = (float *)(smem + ASZ);
#pragma unroll
            for (int v = 0; v < NBV; ++v) {
                const int f = tid + 256 * v;
                if (f < NBT) *(float4 *)&sB[(f >> 3) * LDF + 4 * (f & 7)] = mask4(rwf[v], wval[v]);
            }
        } else {
            uint16_t *sB = (uint16_t *)(smem + ASZ);
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int v = 0; v < NBV; ++v) {
                    const int f = tid + 256 * v;
                    const uint4 w = rwh[q * NBV + v];
                    if (f < NBT)
                        *(uint4 *)&sB[q * LBN * LDH + (f >> 2) * LDH + 8 * lds_chunk(f >> 2, f & 3)] =
                            make_uint4(w.x & wval[v], w.y & wval[v], w.z & wval[v], w.w & wval[v]);
                }
        }
    };

    f32x4 acc[WI][WJ];
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (DMA) {
        // per lane: the 16-byte chunk it copies in each of the wave's 1 KB
        // blocks.  Activations: block b = 4 wave + j holds rows 8 b .. 8 b + 7,
        // chunk c of row r at position c ^ (r & 7).  Weights: block (part q,
        // 2 wave + j) holds rows 16 (2 wave + j) .. + 15, chunk c at
        // lds_chunk(r, c).  Rows are clamped as in the register path; rows
        // that do not exist or are padding only feed accumulator rows that
        // the epilogue never reads.
        int64_t da1[4], da2[4], dw[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 8 * (4 * wave + j) + (lane >> 3);
            const int c = (lane & 7) ^ (r & 7);
            const int64_t row = m0 + r;
            const int lr = TP > 1 ? r % TP : 0;
            const bool pad = TP > 1 && lr > a.n3 + 1;
            int64_t rr = m0;
            if (row < a.rows) rr = pad ? row - (lr - (a.n3 + 1)) : row;
            da1[j] = rr * a.lda1 + 4 * c;
            da2[j] = rr * a.lda2 + 4 * c;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int r = 16 * (2 * wave + j) + (lane >> 2);
            const int c = lds_chunk(r, lane & 3);
            const int o = n0 + r;
            dw[j] = (int64_t)(o < a.nout ? o : n0) * a.ldw + 8 * c;
        }
        auto dma = [&](int kt, int sgi) {
            const int kb = kt * LBK;
            unsigned char *stg = smem + sgi * STG;
            const float *base = kb < a.K1 ? A1 + kb : A2 + (kb - a.K1);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                copy16_to_lds(base + (kb < a.K1 ? da1[j] : da2[j]), stg + (4 * wave + j) * 1024);
            const uint16_t *W = (const uint16_t *)a.W + kb;
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    copy16_to_lds(W + (int64_t)q * a.wpart + dw[j], stg + AST + q * LBN * LBK * 2 + (2 * wave + j) * 1024);
        };
        if (ktiles > 0) dma(0, 0);
        const int ar = wm * 16 * WI + (lane & 15), br = wn * 16 * WJ + (lane & 15);
        const int ko = 8 * lds_chunk(lane & 15, lane >> 4);
        const int h = lane >> 4, sw = lane & 7;          // rows ar + 16 i share bits 0-2 with lane
        for (int kt = 0; kt < ktiles; ++kt) {
            wait_copies();                           // this lane's copies of step kt have landed
            __syncthreads();                         // everyone's have; step kt - 1's stage is free
            // every fragment of step kt is read into registers before the
            // copies of step kt + 1 are issued, so no read of this stage
            // has to wait for those copies
            const unsigned char *stg = smem + (kt & 1) * STG;
            const float *sA = (const float *)stg;
            const uint16_t *sB = (const uint16_t *)(stg + AST);
            float4 xa[WI][2];
            bf16x8 ha[NA][WI], hb[NW][WJ];
#pragma unroll
            for (int i = 0; i < WI; ++i)
                if (i < LIVE || TP != 64) {
                    const float *rowp = sA + (ar + 16 * i) * LBK;
                    xa[i][0] = *(const float4 *)(rowp + 4 * ((2 * h) ^ sw));
                    xa[i][1] = *(const float4 *)(rowp + 4 * ((2 * h + 1) ^ sw));
                }
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int j = 0; j < WJ; ++j) hb[q][j] = *(const bf16x8 *)&sB[q * LBN * LDH + (br + 16 * j) * LDH + ko];
            if (kt + 1 < ktiles) dma(kt + 1, (kt + 1) & 1);
            // split and multiply at raised wave priority: this wave's matrix
            // instructions issue ahead of the other workgroup's on the SIMD,
            // whose fragment reads and copies then fill the gaps
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < WI; ++i)
                if (i < LIVE || TP != 64) {
                    bf16x8 hp[NA];
                    split_fragment<NA>(xa[i][0], xa[i][1], hp);
#pragma unroll
                    for (int q = 0; q < NA; ++q) ha[q][i] = hp[q];
                }
            split_products<NA, NW, TP == 64 ? LIVE : WI, WI, WJ>(ha, hb, acc);
            sched_split_products<NA, NW, TP == 64 ? LIVE : WI, WJ>();
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
            const float *sA = (const float *)smem, *sB = (const float *)(smem + ASZ);
#pragma unroll
            for (int kk = 0; kk < LBK / 4; ++kk) {
                float fa[WI], fb[WJ];
#pragma unroll
                for (int i = 0; i < WI; ++i)
                    if (i < LIVE || TP != 64) fa[i] = sA[(ar + 16 * i) * LDF + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int j = 0; j < WJ; ++j) fb[j] = sB[(br + 16 * j) * LDF + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int i = 0; i < WI; ++i)
#pragma unroll
                    for (int j = 0; j < WJ; ++j)
                        if (i < LIVE || TP != 64)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        } else {
            const uint16_t *sA = (const uint16_t *)smem, *sB = (const uint16_t *)(smem + ASZ);
            const int ko = 8 * lds_chunk(lane & 15, lane >> 4);   // rows ar + 16 i, br + 16 j share bits 0-3 with lane
            bf16x8 ha[NA][WI], hb[NW][WJ];
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int i = 0; i < WI; ++i)
                    if (i < LIVE || TP != 64)
                        ha[q][i] = *(const bf16x8 *)&sA[q * LBM * LDH + (ar + 16 * i) * LDH + ko];
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int j = 0; j < WJ; ++j) hb[q][j] = *(const bf16x8 *)&sB[q * LBN * LDH + (br + 16 * j) * LDH + ko];
            split_products<NA, NW, TP == 64 ? LIVE : WI, WI, WJ>(ha, hb, acc);
        }
    }
    }

    // ---- epilogue through LDS: the pre-activation tile replaces the operand
    //      stage.  Work item = (electron, 4 columns, 16 rows): 256 items per
    //      tile for TP = 16 / 32 / 64, float4 loads and stores, rows unrolled.
    //      Pass 1: z = X + P (+ b on the value row) back into LDS and the
    //      partial Laplacian source sum_c dz_c^2 of the item's rows; pass 2:
    //      value, tangent and Laplacian rows plus the residual.
    const float *__restrict__ Pw = a.Pw;
    const float *__restrict__ bias = a.bias;
    const float *__restrict__ Hin = a.A1;
    float *__restrict__ Hout = a.Hout;
    const int n3 = a.n3, tl = n3 + 1;
    const int64_t rows_here = a.rows - m0 < LBM ? a.rows - m0 : LBM;
    float *sX = (float *)smem;
    auto f4add = [](float4 u, float4 v) { return make_float4(u.x + v.x, u.y + v.y, u.z + v.z, u.w + v.w); };
    // park the accumulators: the pre-activation tile replaces the operand stage
    auto park = [&]() {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
            for (int j = 0; j < WJ; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    sX[(wm * 16 * WI + 16 * i + 4 * (lane >> 4) + e) * XS + wn * 16 * WJ + 16 * j + (lane & 15)] =
                        acc[i][j][e];
        __syncthreads();
    };
    if constexpr (TP == 1) {
        // a thread keeps one column quad and walks 16 rows (8 apart); the
        // per-walker rows are requested before parking, the residual rows
        // right after, so both latencies overlap other work
        constexpr int CQN = LBN / 4, RS = 256 / CQN, NR = LBM / RS;   // rows r0 + RS it, it < NR
        constexpr int HB = NR > 8 ? 8 : NR;                               // residual rows per batch
        const int cq = tid % CQN, r0 = tid / CQN;
        const int col = n0 + 4 * cq;
        const bool colreal = col < a.w1;
        const int colc = colreal ? col : 0;
        const uint32_t cm = colreal ? 0xffffffffu : 0u;
        const float4 bb = mask4(*(const float4 *)(bias + colc), cm);
        float4 pv[NR];
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            const int r = r0 + RS * it;
            const int64_t R = m0 + (r < rows_here ? r : 0);
            pv[it] = *(const float4 *)(Pw + (R / a.N) * a.w1 + colc);
        }
        park();
#pragma unroll
        for (int h = 0; h < NR / HB; ++h) {
            float4 rv[HB];
#pragma unroll
            for (int u = 0; u < HB; ++u) {
                const int r = r0 + RS * (HB * h + u);
                const int64_t R = m0 + (r < rows_here ? r : 0);
                rv[u] = a.resid ? *(const float4 *)(Hin + R * a.lda1 + colc) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < HB; ++u) {
                const int r = r0 + RS * (HB * h + u);
                const float *x = sX + r * XS + 4 * cq;
                const float4 p4 = pv[HB * h + u];
                float4 y = make_float4(tanhf((x[0] + p4.x) + bb.x), tanhf((x[1] + p4.y) + bb.y),
                                       tanhf((x[2] + p4.z) + bb.z), tanhf((x[3] + p4.w) + bb.w));
                y = mask4(f4add(y, rv[u]), cm);
                if (r < rows_here && col < a.W1p) {
                    *(float4 *)(Hout + (m0 + r) * a.ldh_out + col) = y;
                    if (a.Gout) *(float4 *)(sX + r * XS + 4 * cq) = y;
                }
            }
        }
    } else if constexpr (LBN == 128) {
        constexpr int QPR = TP / 16;                   // 16-row chunks per electron
        float4 *srcp = (float4 *)(smem + XSZ);         // [256] partial sources
        const int q = tid;
        const int el = q / (32 * QPR), rem = q % (32 * QPR);
        const int cq = rem / QPR, rc = rem % QPR;
        const int col = n0 + 4 * cq;
        const int64_t Rb = m0 + (int64_t)el * TP;
        const bool live = (int64_t)el * TP < rows_here && col < a.W1p;
        const bool real = live && col < a.w1;
        float *xc = sX + (el * TP) * XS + 4 * cq;
        // the item's per-walker rows and residual rows are requested before
        // the accumulators are parked, so their latency overlaps the parking
        float4 p[16], r4[16];
        float4 b4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (real) {
            const int64_t w = (Rb / TP) / a.N;
            const float *pw = Pw + (w * TP) * (int64_t)a.w1 + col;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int t = 16 * rc + u;
                p[u] = t <= tl ? *(const float4 *)(pw + (int64_t)t * a.w1) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            if (rc == 0) b4 = *(const float4 *)(bias + col);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = 16 * rc + u;
            r4[u] = real && a.resid && t <= tl ? *(const float4 *)(Hin + (Rb + t) * a.lda1 + col)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        park();
        float4 src = make_float4(0.f, 0.f, 0.f, 0.f);
        if (real) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int t = 16 * rc + u;
                float *x = xc + t * XS;
                float4 z = make_float4(x[0] + p[u].x, x[1] + p[u].y, x[2] + p[u].z, x[3] + p[u].w);
                if (t == 0) z = f4add(z, b4);              // (X + P) + b, as the separate epilogue
                x[0] = z.x; x[1] = z.y; x[2] = z.z; x[3] = z.w;
                if (t >= 1 && t <= n3) {
                    src.x += z.x * z.x; src.y += z.y * z.y; src.z += z.z * z.z; src.w += z.w * z.w;
                }
            }
        }
        // with one item per (electron, column quad) the item's own partial
        // source is the whole source: no exchange through LDS
        if constexpr (QPR > 1) {
            srcp[q] = src;
            __syncthreads();
        }
        float y0[4], dd[4], lap[4];
        if (live) {
            float4 s4 = QPR > 1 ? make_float4(0.f, 0.f, 0.f, 0.f) : src;
#pragma unroll
            for (int k = 0; k < QPR; ++k)
                if constexpr (QPR > 1) s4 = f4add(s4, srcp[el * 32 * QPR + cq * QPR + k]);
            const float *z0 = xc, *zl = xc + tl * XS;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                y0[c] = tanhf(z0[c]);
                dd[c] = 1.f - y0[c] * y0[c];
                const float sc = c == 0 ? s4.x : (c == 1 ? s4.y : (c == 2 ? s4.z : s4.w));
                lap[c] = dd[c] * zl[c] - 2.f * y0[c] * dd[c] * sc;
            }
        }
        // rows 0 and tl of an electron are read by all QPR threads of its
        // column group before any of them parks its outputs over them
        if constexpr (QPR > 1) {
            if (a.Gout) __syncthreads();
        }
        if (live) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int t = 16 * rc + u;
                const float *x = xc + t * XS;
                float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
                if (real && t <= tl) {
                    if (t == 0) y = make_float4(y0[0], y0[1], y0[2], y0[3]);
                    else if (t < tl) y = make_float4(dd[0] * x[0], dd[1] * x[1], dd[2] * x[2], dd[3] * x[3]);
                    else y = make_float4(lap[0], lap[1], lap[2], lap[3]);
                    y = f4add(y, r4[u]);
                }
                if (t <= tl) *(float4 *)(Hout + (Rb + t) * a.ldh_out + col) = y;   // padding rows are not written
                if (a.Gout) *(float4 *)(xc + t * XS) = y;
            }
        }
    }
    // spin means of the finished rows for the next layer (whole walkers per
    // tile): item = (walker, row t, spin, 4 columns)
    if (a.Gout) {
        __syncthreads();
        const int wpt = LBM / (a.N * TP);                 // walkers in this tile
        const int nd = a.N - a.nu;
        const float iu = a.nu > 0 ? 1.f / a.nu : 0.f, id = nd > 0 ? 1.f / nd : 0.f;
        const int64_t ldg = 2 * (int64_t)a.W1p;
        for (int q = tid; q < wpt * TP * 2 * (LBN / 4); q += 256) {
            const int c4 = q % (LBN / 4), rest = q / (LBN / 4);
            const int sp = rest % 2, wt = rest / 2;       // wt = walker-in-tile * TP + t
            const int wl = wt / TP, t = wt % TP;
            const int64_t wg = m0 / ((int64_t)a.N * TP) + wl;
            if ((int64_t)(wl + 1) * a.N * TP > rows_here || n0 + 4 * c4 >= a.W1p) continue;
            if (t > a.n3 + 1) continue;                   // padding rows: never read
            const int j0 = sp ? a.nu : 0, j1 = sp ? a.N : a.nu;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int j = j0; j < j1; ++j) v = f4add(v, *(const float4 *)(sX + ((wl * a.N + j) * TP + t) * XS + 4 * c4));
            const float sc = sp ? id : iu;
            *(float4 *)(a.Gout + (wg * TP + t) * ldg + sp * a.W1p + n0 + 4 * c4) =
                make_float4(v.x * sc, v.y * sc, v.z * sc, v.w * sc);
        }
    }
}

// Value rows (TP = 1) in a grid too small to fill the CUs, split-BF16 modes:
// 32 x 32 output tiles whose reduction steps are split over the four waves
// (in contiguous quarters, partial tiles summed in LDS in wave order), then
// the value epilogue of k_stream_layer: y = tanh((x + P_walker) + b)
// (+ h^l), zero past w1, and the next layer's spin means when a 32-row tile
// holds whole walkers (N divides 32).
template <int MODE>
__global__ __launch_bounds__(256) void k_stream_value_splitk(LayerArgs a)
{
    constexpr int NA = act_parts(MODE), NW = weight_parts(MODE);
    static_assert(MODE != GEMM_F32, "split-BF16 modes");
    __shared__ float red[4][32][33];
    __shared__ __attribute__((aligned(16))) float sy[32][36];
    auto f4add = [](float4 u, float4 v) { return make_float4(u.x + v.x, u.y + v.y, u.z + v.z, u.w + v.w); };
    const int tid = threadIdx.x;
    const int64_t nrb = (a.rows + 31) / 32;
    const int64_t m0 = (blockIdx.x % nrb) * 32;
    const int n0 = (int)(blockIdx.x / nrb) * 32;
    if (n0 >= a.W1p) return;
    const int64_t rows_here = a.rows - m0 < 32 ? a.rows - m0 : 32;
    // epilogue item: row r, column quad cq; its per-walker row, bias and
    // residual are requested before the reduction
    const int r = tid >> 3, cq = tid & 7;
    const int col = n0 + 4 * cq;
    const bool colreal = col < a.w1;
    const int colc = colreal ? col : 0;
    const uint32_t cm = colreal ? 0xffffffffu : 0u;
    const int64_t R = m0 + (r < rows_here ? r : 0);
    const float4 bb = mask4(*(const float4 *)(a.bias + colc), cm);
    const float4 p4 = *(const float4 *)(a.Pw + (R / a.N) * a.w1 + colc);
    const float4 rv = a.resid ? *(const float4 *)(a.A1 + R * a.lda1 + colc) : make_float4(0.f, 0.f, 0.f, 0.f);
    f32x4 acc[2][2];
    splitk_accumulate<NA, NW>(a.A1, a.lda1, a.K1, a.A2, a.lda2, a.K2, (const uint16_t *)a.W, a.wpart, a.ldw, a.nout,
                          a.rows, m0, n0, [](int64_t row) { return row; }, acc);
    splitk_park(acc, red);
    float x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        x[e] = ((red[0][r][4 * cq + e] + red[1][r][4 * cq + e]) + red[2][r][4 * cq + e]) + red[3][r][4 * cq + e];
    float4 y = make_float4(tanhf((x[0] + p4.x) + bb.x), tanhf((x[1] + p4.y) + bb.y), tanhf((x[2] + p4.z) + bb.z),
                           tanhf((x[3] + p4.w) + bb.w));
    y = mask4(f4add(y, rv), cm);
    if (r < rows_here && col < a.W1p) *(float4 *)(a.Hout + (m0 + r) * a.ldh_out + col) = y;
    if (a.Gout) {
        *(float4 *)&sy[r][4 * cq] = y;
        __syncthreads();
        const int wpt = 32 / a.N;
        const int nd = a.N - a.nu;
        const float iu = a.nu > 0 ? 1.f / a.nu : 0.f, id = nd > 0 ? 1.f / nd : 0.f;
        const int64_t ldg = 2 * (int64_t)a.W1p;
        for (int q = tid; q < wpt * 2 * 8; q += 256) {
            const int c4 = q & 7, sp = (q >> 3) & 1, wl = q >> 4;
            if ((int64_t)(wl + 1) * a.N > rows_here || n0 + 4 * c4 >= a.W1p) continue;
            const int j0 = sp ? a.nu : 0, j1 = sp ? a.N : a.nu;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int j = j0; j < j1; ++j) v = f4add(v, *(const float4 *)&sy[wl * a.N + j][4 * c4]);
            const float sc = sp ? id : iu;
            *(float4 *)(a.Gout + (m0 / a.N + wl) * ldg + sp * a.W1p + n0 + 4 * c4) =
                make_float4(v.x * sc, v.y * sc, v.z * sc, v.w * sc);
        }
    }
}

// Default path for the stream layers in every MFMA mode whose row layout it
// supports; the separate product + epilogue kernels remain for the others
// (and for the backward pass, which keeps the tanh outputs).
bool g_use_fused_layer = true;

bool stream_layer_supported(int mode, int TR, int w1, int W1p)
{
    return g_use_fused_layer && mode != GEMM_F64 && W1p <= 256 && w1 % 4 == 0 &&
           (TR == 1 || TR == 16 || TR == 32 || TR == 64);
}

// Split-BF16 modes with 128-column tiles stage their operands by direct
// global-to-LDS copies (two stages); the register-staged path stays for
// FP32, the 32-column value tiles, and as the tuning switch "layer_dma" = 0.
// Both give bitwise the same results.
bool g_layer_dma = true;

template <int MODE, bool DMA>
static void launch_tiles(const LayerArgs &a, int TR, dim3 grid, hipStream_t st)
{
    switch (TR) {
    case 1: hipLaunchKernelGGL((k_stream_layer<MODE, 1, 128, 1, DMA>), grid, dim3(256), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_stream_layer<MODE, 16, 128, 1, DMA>), grid, dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_stream_layer<MODE, 32, 128, 2, DMA>), grid, dim3(256), 0, st, a); break;
    default:
        // rows value .. Laplacian (3N + 2) within the first three row blocks
        if (a.n3 + 2 <= 48) hipLaunchKernelGGL((k_stream_layer<MODE, 64, 128, 3, DMA>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_stream_layer<MODE, 64, 128, 4, DMA>), grid, dim3(256), 0, st, a);
        break;
    }
}

template <int MODE>
static void launch_mode(const LayerArgs &a, int TR, hipStream_t st)
{
    const int64_t nrb = (a.rows + LBM - 1) / LBM;
    const int64_t blocks = xcd_grid(nrb, (a.W1p + 127) / 128);
    // value rows in a grid too small to fill the CUs: in the split-BF16 modes
    // 32 x 32 tiles with the reduction split over the waves while there are
    // fewer 128 x 32 tiles than CUs, else 32-column tiles, so each
    // workgroup's reduction steps carry a quarter of the matrix work
    if constexpr (MODE != GEMM_F32) {
        if (TR == 1 && g_gemm_splitk && !g_splitk_suppressed && a.K1 % 32 == 0 && a.K2 % 32 == 0 && (!a.Gout || 32 % a.N == 0) &&
            nrb * ((a.W1p + 31) / 32) < 256) {
            dim3 grid((unsigned)(((a.rows + 31) / 32) * ((a.W1p + 31) / 32)));
            hipLaunchKernelGGL((k_stream_value_splitk<MODE>), grid, dim3(256), 0, st, a);
            return;
        }
    }
    if (TR == 1 && blocks <= 512) {
        dim3 grid((unsigned)(nrb * ((a.W1p + 31) / 32)));
        hipLaunchKernelGGL((k_stream_layer<MODE, 1, 32, 1, false>), grid, dim3(256), 0, st, a);
        return;
    }
    if constexpr (MODE != GEMM_F32) {
        if (g_layer_dma) {
            launch_tiles<MODE, true>(a, TR, dim3((unsigned)blocks), st);
            return;
        }
    }
    launch_tiles<MODE, false>(a, TR, dim3((unsigned)blocks), st);
}

void launch_stream_layer(int mode, const LayerArgs &a, int TR, hipStream_t st)
{
    if (a.rows <= 0) return;
    switch (mode) {
    case GEMM_F32: launch_mode<GEMM_F32>(a, TR, st); break;
    default: with_split_mode(mode, [&](auto m) { launch_mode<decltype(m)::value>(a, TR, st); }); break;
    }
}

}  // namespace fn
