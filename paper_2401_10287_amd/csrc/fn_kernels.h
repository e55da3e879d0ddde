// fn_kernels.h -- launchers of the network kernels (fn_net.hip), the backward
// pass (fn_backward.hip) and the Monte Carlo kernels (fn_mc.hip).
#pragma once
#include "fn_internal.h"

namespace fn {

// Packing of the forward operands from the flat parameter vector: one
// segment per layer (kind 0: per-electron block Wx into d0, per-walker block
// Wg into d1) and per spin head (kind 1: Wh into d0), in the product's
// operand type (mode); segment q covers elements [begin, begin + count).
// Kind 2: FP32 pair block of one pair layer in the matrix-core pair
// kernel's layout (transposed weights Wt[wc][ks] from off, then the bias
// [wc] from off2) into d0.
// kind 0: a layer's Wx / Wg operand blocks; 1: a head block; 2: a pair
// block; 3: a plain copy of count parameters from off, rounded to BF16 (the
// layer weights the backward of the BF16-weight modes multiplies with).
// round: layer weights are taken as their BF16 roundings before packing.
struct PackSeg {
    int64_t begin, count, off, off2;
    int kind, mode, mode2, dh, dp, w1, HWl, GWl, kn, W1p, w2, wc, ks;   // mode2: Wg of a layer block
    int round;
    int bbegin;     // first workgroup of the segment (set by launch_pack)
    void *d0, *d1;
};
struct PackList {
    int n;
    PackSeg seg[4 * FN_MAX_LAYERS + 2];
};
static_assert(sizeof(PackList) < 4000, "kernel argument");
template <typename T>
void launch_pack(const T *theta, const PackList &pl, hipStream_t st);
// G (or nullptr): also the first layer's spin means of the features, in the
// layout and arithmetic of launch_spin_mean
template <typename T>
void launch_features(const Sys &s, const double *x, int64_t B, int TR, int HW0, int64_t ldh, T *H, T *G,
                     hipStream_t st);
size_t pair_stream_lds(const Sys &s, bool fl, size_t elem);
// Matrix-core pair kernel layout of the pair weights: per pair layer l the
// transposed weights Wt[wc][KP_l + 4] (wc = w2 rounded up to 16, KP_l = d_p
// of layer l rounded up to 16), then the bias [wc]; pair_mfma_woff(s, l) is
// the float offset of layer l's block, pair_mfma_woff(s, L - 1) the total.
__host__ __device__ inline int pair_mfma_kp(const Sys &s, int l) { return round_up(layer_dp(s, l), 16); }
__host__ __device__ inline int pair_mfma_woff(const Sys &s, int l)
{
    const int wc = round_up(s.w2, 16);
    int o = 0;
    for (int q = 0; q < l; ++q) o += wc * (pair_mfma_kp(s, q) + 4) + wc;
    return o;
}
// wpair: the packed pair weights above (FP32 parameters), or nullptr
template <typename T>
void launch_pair_stream(const Sys &s, const double *x, const T *theta, const ParamLayout &P, int64_t B, int TR,
                        bool fl, int64_t ldg, int64_t gi_layer_stride, int GW0, int GW1, const float *wpair, T *GI,
                        hipStream_t st);
template <typename T>
void launch_spin_mean(const T *H, int64_t ldh, int64_t B, int N, int nu, int TR, int dh, int HWl, T *G,
                      hipStream_t st);
template <typename T>
void launch_layer_epi(const T *X, const T *Pw, const T *bias, const T *Hin, T *Hout, int64_t ldh, int64_t B, int N,
                      int TR, int n3, int w1, int W1p, int resid, bool fl, T *Tout, hipStream_t st);
template <typename T>
void launch_envelope(const Sys &s, const double *x, const T *theta, int64_t gof, int64_t piof, int64_t sigof, int sp,
                     const T *O, int64_t ldo, int64_t B, int TR, bool fl, double *Phi, hipStream_t st);
size_t det_lds(int n, int n3, bool fl, size_t elem);
size_t orbdet_lds(int n, bool fl);
// Per-spin operands of the fused orbital / envelope / determinant stage:
// parameter offsets of g, pi and Sigma, and the head output O with its
// leading dimension.  One launch covers both spins when they have the same
// size (the kernels take the spin from the block index).
template <typename T>
struct OrbSpins {
    int64_t gof0, gof1, piof0, piof1, sigof0, sigof1, ldo0, ldo1;
    const T *O0, *O1;
};
template <typename T>
void launch_orbdet(const Sys &s, const double *x, const T *theta, const OrbSpins<T> &S, int64_t B, int TR, bool fl,
                   double *DR, int rec, hipStream_t st);
void launch_det(const double *Phi, int64_t B, int K, int n, int TR, int n3, int sp, bool fl, double *DR, int rec,
                hipStream_t st);
// Metropolis acceptance folded into the value-only combine of the proposal:
// walker w keeps x'[w] (and log|psi'|) iff log|psi'| is finite and
// log u[w] <= 2 (log|psi'| - log_abs[w]); x == nullptr: no acceptance.
struct AcceptArgs {
    double *x;               // current positions [B][3N], updated in place
    const double *xp;        // proposed positions [B][3N]
    const double *u;         // uniforms [B]
    double *log_abs;         // current log|psi| [B], updated in place
    int32_t *n_accept;       // per-walker acceptance counters [B] or nullptr
};
void launch_combine(const Sys &s, const double *x, const double *DR, int rec, int64_t B, double vnn, double *log_abs,
                    int8_t *sign, double *e_loc, double *parts, bool fl, const AcceptArgs &acc, hipStream_t st);
// Value form with both spins of 1..8 electrons and K <= 32: the orbital /
// determinant stage and the combine (with the acceptance) in one launch;
// results equal to launch_orbdet followed by launch_combine.  false (nothing
// launched) for other shapes.
template <typename T>
bool launch_orbdet_combine(const Sys &s, const double *x, const T *theta, const OrbSpins<T> &S, int64_t B, int TR,
                           double *log_abs, int8_t *sign, const AcceptArgs &acc, hipStream_t st);

// backward (fn_backward.hip)
size_t det_backward_lds(int n);
void launch_det_backward(const double *Phi, const double *DR, const double *coeff, int64_t B, int K, int n, int sp,
                         int nu, int nd, int rec, double *GA, hipStream_t st);
// Eq. 5: GA = scale (Phi - target) per (walker, determinant, orbital, electron)
// and lsum[w] += sum of squared differences of walker w
void launch_pretrain_adjoint(const double *Phi, const double *target, int64_t B, int K, int n, double scale, double *GA,
                             double *lsum, hipStream_t st);
// loss = sum_w (lsum[w] + lsum[B + w]) / B
void launch_pretrain_loss(const double *lsum, int64_t B, double *loss, hipStream_t st);
template <typename T>
void launch_env_backward(const Sys &s, const double *x, const T *theta, int64_t gof, int64_t piof, int64_t sigof,
                         int sp, const T *O, int64_t ldo, const double *GA, int64_t B, int KNp, T *Ga, T *EP,
                         hipStream_t st);
template <typename T>
void launch_bwd_gz(const T *Gy, const T *Tt, int64_t B, int N, int w1, T *Gz, T *SGz, hipStream_t st);
template <typename T>
void launch_bwd_gh(const T *Gh, const T *Gy, const T *Gg, int64_t B, int N, int nu, int dh, int w1, int resid, T *Gout,
                   hipStream_t st);
size_t pair_backward_lds(const Sys &s, size_t elem);
int pair_backward_wb(const Sys &s, size_t elem);      // (walker, electron) rows per vector-kernel workgroup
// Pair-stream adjoint: writes one row of npp weight-gradient shares per
// workgroup into PP and returns the number of rows written.  wpair: the pair
// weights packed for the matrix-core pair kernel (FP32 parameters), or
// nullptr for the vector kernel.
template <typename T>
int64_t launch_pair_backward(const Sys &s, const double *x, const T *theta, const ParamLayout &P, int64_t B,
                             const T *GGI, int64_t ldg, int64_t gg_layer_stride, const float *wpair, T *PP, int64_t npp,
                             hipStream_t st);
int max_splits();
template <typename T>
void launch_tn(const T *X, int64_t ldx, int NA, const T *Y, int64_t ldy, int NB, int64_t R, int64_t per,
               int64_t stride, int64_t off, T *part, double *acc, int64_t acc_off, int64_t lda_out, hipStream_t st);
template <typename T>
void launch_colsum(const T *in, int64_t ld, int C, int64_t R, T *part, double *acc, int64_t off, int env_map,
                   int64_t off2, hipStream_t st);
void launch_zero_f64(double *p, int64_t n, hipStream_t st);
template <typename T>
void launch_grad_out(const double *acc, int64_t n, T *grad, hipStream_t st);
template <typename T>
void launch_pack_head_bwd(const T *theta, int64_t woff, int w1, int kn, int KNp, bool round, T *Wb, hipStream_t st);

// Monte Carlo
void launch_propose(const double *x, int64_t B, int n3, double sigma, uint64_t seed, uint64_t step, uint32_t stream_id,
                    const double *z_ext, const double *u_ext, double *xp, double *u, hipStream_t st);
// per-job generator state of a grouped Metropolis call: job q owns walkers
// [w0[q], w0[q + 1]) of the group, key (k0, k1), step counter, stream id
struct GroupTable {
    int n;
    int64_t w0[FN_MAX_GROUP_JOBS + 1];
    uint32_t k0[FN_MAX_GROUP_JOBS], k1[FN_MAX_GROUP_JOBS], step[FN_MAX_GROUP_JOBS], stream[FN_MAX_GROUP_JOBS];
};
void launch_propose_group(const double *x, int64_t B, int n3, double sigma, const GroupTable &g, double *xp,
                          double *u, hipStream_t st);
void launch_energy_stats(const double *e_loc, int64_t B, double *stats, double *coeff, hipStream_t st);

}  // namespace fn
