// fn_backward.hip -- reverse pass of log|psi| with respect to the parameters,
// weighted over walkers: grad = sum_p c_p d log|psi_p| / d theta.  With
// c_p = 2 (E_p - mean E) / B this is the training gradient of Eq. 6 of the
// paper; any other weights give the vector-Jacobian product of log|psi|.
//
// Adjoints, from the output down (value rows only, stream activations of the
// one-electron layers saved by the forward pass, pair-stream activations
// recomputed per electron):
//   log|psi| = log|sum_k s_k exp(l_k)|:   d/d l_k = omega_k = psi_k / psi
//   l_k = log|det A_k|:                   d/d A_k = A_k^-T
//   A[i][j] = a_i(r_j) env_i(r_j):        d/d a = G env, d/d env = G a
//   a = w . h_j^L + g, env = sum_m pi_m exp(-|Sigma_m (r_j - R_m)|)
//   h^{l+1} = tanh(z) (+ h^l), z = [h_i, g_up, g_dn, g_i_up, g_i_dn] V + b
//   pair layers h_ij^{l+1} = tanh(W2^T h_ij^l + c2) (+ h_ij^l), g_i = spin mean
// Weight gradients are sums over walkers x electrons of outer products; they
// are formed as split row reductions whose partial sums are added in a fixed
// order, so the result does not depend on scheduling.
#include <type_traits>

#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

namespace {

__device__ inline double wsum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

unsigned gridn(int64_t n, int bs = 256)
{
    int64_t g = (n + bs - 1) / bs;
    if (g > (1 << 20)) g = 1 << 20;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

// ---------------------------------------------------------------------------
// determinant adjoint: GA[w][k][i][j] = c_w omega_k (A_k^-1)[j][i]; one wave64
// per (walker, determinant) of one spin.  Walkers on a node (psi = 0) and
// singular determinants contribute nothing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_det_backward(const double *Phi, const double *DR, const double *coeff,
                                                     int64_t B, int K, int n, int sp, int nu, int nd, int rec,
                                                     double *GA)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    double *LU = (double *)smem_raw;
    double *Inv = LU + n * n;
    int *perm = (int *)(Inv + n * n);
    __shared__ double s_scale;
    __shared__ int s_sing;
    const int lane = threadIdx.x;
    const int64_t w = blockIdx.x / K;
    const int k = (int)(blockIdx.x % K);
    if (w >= B) return;
    const int64_t nn = (int64_t)n * n;
    double *out = GA + (w * K + k) * nn;
    if (lane == 0) {
        const double *ru = DR + (w * 2 + 0) * (int64_t)K * rec, *rd = DR + (w * 2 + 1) * (int64_t)K * rec;
        double lmax = -INFINITY;
        for (int q = 0; q < K; ++q) {
            double s = (nu > 0 ? ru[q * rec] : 1.0) * (nd > 0 ? rd[q * rec] : 1.0);
            double l = (nu > 0 ? ru[q * rec + 1] : 0.0) + (nd > 0 ? rd[q * rec + 1] : 0.0);
            if (s != 0.0 && l > lmax) lmax = l;
        }
        double S = 0.0, mine = 0.0;
        if (lmax > -INFINITY)
            for (int q = 0; q < K; ++q) {
                double s = (nu > 0 ? ru[q * rec] : 1.0) * (nd > 0 ? rd[q * rec] : 1.0);
                double l = (nu > 0 ? ru[q * rec + 1] : 0.0) + (nd > 0 ? rd[q * rec + 1] : 0.0);
                double t = s != 0.0 ? s * exp(l - lmax) : 0.0;
                S += t;
                if (q == k) mine = t;
            }
        const bool ok = lmax > -INFINITY && S != 0.0 && S == S;
        s_scale = ok ? coeff[w] * mine / S : 0.0;
        s_sing = 0;
    }
    const double *A = Phi + (w * K + k) * nn;
    for (int q = lane; q < n * n; q += 64) LU[q] = A[q];
    for (int q = lane; q < n; q += 64) perm[q] = q;
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        if (lane == 0) {
            int p = c;
            double best = fabs(LU[c * n + c]);
            for (int r = c + 1; r < n; ++r) {
                double v = fabs(LU[r * n + c]);
                if (v > best) { best = v; p = r; }
            }
            if (best == 0.0) s_sing = 1;
            else if (p != c) {
                for (int q = 0; q < n; ++q) { double t = LU[c * n + q]; LU[c * n + q] = LU[p * n + q]; LU[p * n + q] = t; }
                int t = perm[c]; perm[c] = perm[p]; perm[p] = t;
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
    if (s_sing || s_scale == 0.0) {
        for (int q = lane; q < n * n; q += 64) out[q] = 0.0;
        return;
    }
    // column c of A^-1 = U^-1 L^-1 P e_c, one column per lane
    for (int c = lane; c < n; c += 64) {
        for (int r = 0; r < n; ++r) Inv[r * n + c] = perm[r] == c ? 1.0 : 0.0;
        for (int r = 1; r < n; ++r) {
            double acc = Inv[r * n + c];
            for (int q = 0; q < r; ++q) acc -= LU[r * n + q] * Inv[q * n + c];
            Inv[r * n + c] = acc;
        }
        for (int r = n - 1; r >= 0; --r) {
            double acc = Inv[r * n + c];
            for (int q = r + 1; q < n; ++q) acc -= LU[r * n + q] * Inv[q * n + c];
            Inv[r * n + c] = acc / LU[r * n + r];
        }
    }
    __syncthreads();
    const double sc = s_scale;
    for (int q = lane; q < n * n; q += 64) {
        const int i = q / n, j = q % n;
        out[q] = sc * Inv[j * n + i];
    }
}

// The same for spins of at most NS electrons with one thread per (walker,
// determinant k): the LU factors in registers, the inverse formed one column
// at a time (column c of A^-1 is row c of the output), every operation in the
// order of the wave kernel.
template <int NS>
__global__ __launch_bounds__(256) void k_det_backward_small(const double *Phi, const double *DR, const double *coeff,
                                                            int64_t B, int K, int n, int nu, int nd, int rec,
                                                            double *GA)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= B * K) return;
    const int64_t w = id / K;
    const int k = (int)(id % K);
    const int64_t nn = (int64_t)n * n;
    double *out = GA + (w * K + k) * nn;
    const double *ru = DR + (w * 2 + 0) * (int64_t)K * rec, *rd = DR + (w * 2 + 1) * (int64_t)K * rec;
    double lmax = -INFINITY;
    for (int q = 0; q < K; ++q) {
        const double s = (nu > 0 ? ru[q * rec] : 1.0) * (nd > 0 ? rd[q * rec] : 1.0);
        const double l = (nu > 0 ? ru[q * rec + 1] : 0.0) + (nd > 0 ? rd[q * rec + 1] : 0.0);
        if (s != 0.0 && l > lmax) lmax = l;
    }
    double S = 0.0, mine = 0.0;
    if (lmax > -INFINITY)
        for (int q = 0; q < K; ++q) {
            const double s = (nu > 0 ? ru[q * rec] : 1.0) * (nd > 0 ? rd[q * rec] : 1.0);
            const double l = (nu > 0 ? ru[q * rec + 1] : 0.0) + (nd > 0 ? rd[q * rec + 1] : 0.0);
            const double t = s != 0.0 ? s * exp(l - lmax) : 0.0;
            S += t;
            if (q == k) mine = t;
        }
    const bool ok = lmax > -INFINITY && S != 0.0 && S == S;
    const double sc = ok ? coeff[w] * mine / S : 0.0;
    double LU[NS][NS];
    int perm[NS];
    const double *A = Phi + (w * K + k) * nn;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        perm[r] = r;
#pragma unroll
        for (int c = 0; c < NS; ++c) LU[r][c] = r < n && c < n ? A[r * n + c] : 0.0;
    }
    bool sing = false;
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        if (c >= n || sing) continue;
        int p = c;
        double best = fabs(LU[c][c]);
#pragma unroll
        for (int r = c + 1; r < NS; ++r) {
            if (r >= n) continue;
            const double v = fabs(LU[r][c]);
            if (v > best) { best = v; p = r; }
        }
        if (best == 0.0) { sing = true; continue; }
        if (p != c) {
            // row swap with a register-indexed partner: select over the rows
#pragma unroll
            for (int r = c + 1; r < NS; ++r) {
                if (r == p) {
#pragma unroll
                    for (int q = 0; q < NS; ++q) { const double t = LU[c][q]; LU[c][q] = LU[r][q]; LU[r][q] = t; }
                    const int t = perm[c]; perm[c] = perm[r]; perm[r] = t;
                }
            }
        }
        const double ip = 1.0 / LU[c][c];
#pragma unroll
        for (int r = c + 1; r < NS; ++r)
            if (r < n) LU[r][c] *= ip;
#pragma unroll
        for (int r = c + 1; r < NS; ++r)
#pragma unroll
            for (int cc = c + 1; cc < NS; ++cc)
                if (r < n && cc < n) LU[r][cc] -= LU[r][c] * LU[c][cc];
    }
    if (sing || sc == 0.0) {
        for (int q = 0; q < nn; ++q) out[q] = 0.0;
        return;
    }
    for (int c = 0; c < n; ++c) {
        double v[NS];
#pragma unroll
        for (int r = 0; r < NS; ++r) v[r] = perm[r] == c ? 1.0 : 0.0;
#pragma unroll
        for (int r = 1; r < NS; ++r) {
            if (r >= n) continue;
            double acc = v[r];
#pragma unroll
            for (int q = 0; q < r; ++q) acc -= LU[r][q] * v[q];
            v[r] = acc;
        }
#pragma unroll
        for (int r = NS - 1; r >= 0; --r) {
            if (r >= n) continue;
            double acc = v[r];
#pragma unroll
            for (int q = r + 1; q < NS; ++q)
                if (q < n) acc -= LU[r][q] * v[q];
            v[r] = acc / LU[r][r];
        }
        // out[i][j] = sc (A^-1)[j][i]: column c of A^-1 is row c of out
#pragma unroll
        for (int r = 0; r < NS; ++r)
            if (r < n) out[c * n + r] = sc * v[r];
    }
}

// ---------------------------------------------------------------------------
// envelope / orbital adjoint, one thread per (walker, orbital column):
//   Ga[w n + j][col] = G env                       (adjoint of a = w . h + g)
//   EP[w][col][m][0]   = sum_j G a exp(-q_m)             (pi_m)
//   EP[w][col][m][1+3p+q] = sum_j -G a pi_m exp(-q_m) (Sigma d)_p d_q / q
// and for the isotropic envelope (q_m = |sigma_m| r_m, two partials):
//   EP[w][col][m][1] = sum_j -G a pi_m exp(-q_m) sign(sigma_m) r_m
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_env_backward(Sys s, const double *x, const T *theta, int64_t gof, int64_t piof, int64_t sigof, int sp,
                               const T *O, int64_t ldo, const double *GA, int64_t B, int KNp, T *Ga, T *EP)
{
    const int n = sp == 0 ? s.nu : s.nd, j0 = sp == 0 ? 0 : s.nu;
    const int kn = s.K * n;
    const int64_t total = B * KNp;
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total; id += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(id % KNp);
        const int64_t w = id / KNp;
        if (col >= kn) {
            for (int jj = 0; jj < n; ++jj) Ga[(w * n + jj) * KNp + col] = T(0);
            continue;
        }
        const int k = col / n, io = col % n;
        const double gcol = (double)theta[gof + col];
        // adjoint of a for each electron j of this spin
        for (int jj = 0; jj < n; ++jj) {
            const double *xj = x + (w * s.N + j0 + jj) * 3;
            double env = 0.0;
            for (int m = 0; m < s.M; ++m) {
                const double d0 = xj[0] - s.R[m][0], d1 = xj[1] - s.R[m][1], d2 = xj[2] - s.R[m][2];
                double q;
                if (s.iso) {
                    q = fabs((double)theta[sigof + (int64_t)col * s.M + m]) * sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                } else {
                    const T *Sg = theta + sigof + ((int64_t)col * s.M + m) * 9;
                    double q2 = 0.0;
                    for (int p = 0; p < 3; ++p) {
                        const double v = (double)Sg[3 * p] * d0 + (double)Sg[3 * p + 1] * d1 + (double)Sg[3 * p + 2] * d2;
                        q2 += v * v;
                    }
                    q = sqrt(q2);
                }
                env += (double)theta[piof + (int64_t)col * s.M + m] * exp(-q);
            }
            const double G = GA[((w * s.K + k) * n + io) * n + jj];
            Ga[(w * n + jj) * KNp + col] = (T)(G * env);
        }
        // envelope parameters, summed over the electrons of this walker
        if (s.iso) {
            for (int m = 0; m < s.M; ++m) {
                const double sraw = (double)theta[sigof + (int64_t)col * s.M + m];
                const double sg = fabs(sraw), sgn = sraw < 0.0 ? -1.0 : 1.0;
                const double pim = (double)theta[piof + (int64_t)col * s.M + m];
                double gp = 0.0, gs = 0.0;
                for (int jj = 0; jj < n; ++jj) {
                    const double *xj = x + (w * s.N + j0 + jj) * 3;
                    const double d0 = xj[0] - s.R[m][0], d1 = xj[1] - s.R[m][1], d2 = xj[2] - s.R[m][2];
                    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    const double e = exp(-(sg * r));
                    const double a0 = (double)O[(w * n + jj) * ldo + col] + gcol;
                    const double ga = GA[((w * s.K + k) * n + io) * n + jj] * a0;
                    gp += ga * e;
                    gs -= ga * pim * e * sgn * r;
                }
                T *ep = EP + ((w * kn + col) * s.M + m) * 2;
                ep[0] = (T)gp;
                ep[1] = (T)gs;
            }
            continue;
        }
        for (int m = 0; m < s.M; ++m) {
            const T *Sg = theta + sigof + ((int64_t)col * s.M + m) * 9;
            const double pim = (double)theta[piof + (int64_t)col * s.M + m];
            double gp = 0.0, gs[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int jj = 0; jj < n; ++jj) {
                const double *xj = x + (w * s.N + j0 + jj) * 3;
                const double d[3] = {xj[0] - s.R[m][0], xj[1] - s.R[m][1], xj[2] - s.R[m][2]};
                double sd[3];
                for (int p = 0; p < 3; ++p) sd[p] = (double)Sg[3 * p] * d[0] + (double)Sg[3 * p + 1] * d[1] + (double)Sg[3 * p + 2] * d[2];
                const double q = sqrt(sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2]);
                const double e = exp(-q);
                const double a0 = (double)O[(w * n + jj) * ldo + col] + gcol;
                const double G = GA[((w * s.K + k) * n + io) * n + jj];
                const double ga = G * a0;
                gp += ga * e;
                const double f = -ga * pim * e / q;
                for (int p = 0; p < 3; ++p)
                    for (int qq = 0; qq < 3; ++qq) gs[3 * p + qq] += f * sd[p] * d[qq];
            }
            T *ep = EP + ((w * kn + col) * s.M + m) * 10;
            ep[0] = (T)gp;
            for (int e = 0; e < 9; ++e) ep[1 + e] = (T)gs[e];
        }
    }
}

// ---------------------------------------------------------------------------
// layer adjoints (value rows)
// ---------------------------------------------------------------------------
// Gz = Gy (1 - t^2) per electron row, SGz[w] = sum over the walker's electrons
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_gz(const T *__restrict__ Gy, const T *__restrict__ Tt, int N, int w1,
                                                T *__restrict__ Gz, T *__restrict__ SGz)
{
    const int64_t w = blockIdx.x;
    for (int o = threadIdx.x; o < w1; o += blockDim.x) {
        T acc = T(0);
        for (int i = 0; i < N; ++i) {
            const int64_t r = (w * N + i) * w1 + o;
            const T t = Tt[r];
            const T g = Gy[r] * (T(1) - t * t);
            Gz[r] = g;
            acc += g;
        }
        SGz[w * w1 + o] = acc;
    }
}

// adjoint of h^l: Gh (through V_h) + residual + spin-mean part Gg / n_spin
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_gh(const T *__restrict__ Gh, const T *__restrict__ Gy,
                                                const T *__restrict__ Gg, int N, int nu, int dh, int w1, int resid,
                                                T *__restrict__ Gout)
{
    const int64_t wi = blockIdx.x;
    const int64_t w = wi / N;
    const int i = (int)(wi % N);
    const int sp = i < nu ? 0 : 1;
    const T inv = T(1) / T(sp == 0 ? nu : N - nu);
    for (int u = threadIdx.x; u < dh; u += blockDim.x) {
        T v = Gh[wi * dh + u] + Gg[w * 2 * dh + sp * dh + u] * inv;
        if (resid) v += Gy[wi * w1 + u];
        Gout[wi * w1 + u] = v;
    }
}

// ---------------------------------------------------------------------------
// pair stream adjoint: a workgroup takes WB consecutive (walker, electron i),
// recomputes their pair activations h_ij^l, runs back through the pair layers
// with the adjoints of the spin means g_i^l (GGI, ld ldg, columns [up | dn])
// and writes the summed share of dW2, dc2 of its rows (one PP row per
// workgroup, layout of theta from W2_0 on; rows summed in a fixed order).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_pair_backward(Sys s, const double *x, const T *theta, ParamLayout P, int64_t B,
                                                       const T *GGI, int64_t ldg, int64_t gg_layer_stride, int WB,
                                                       T *PP, int64_t npp)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int wp = s.w2 > 4 ? s.w2 : 4;
    const int N = s.N, L = s.L;
    const int per = (2 * L + 2) * N * wp;     // one (walker, electron) row
    // pair weights and biases (theta from W2_0 on) staged after the rows
    T *Wsm = (T *)smem_raw + (size_t)WB * per;
    const int64_t npw = L > 1 ? P.c2[L - 2] + s.w2 - P.W2[0] : 0;
    for (int64_t q = threadIdx.x; q < npw; q += blockDim.x) Wsm[q] = theta[P.W2[0] + q];
    const int64_t wi0 = (int64_t)blockIdx.x * WB;
    const int nwi = B * N - wi0 < WB ? (int)(B * N - wi0) : WB;
    // per row: Hs [L][N][wp] activations, Ts [L][N][wp] tanh outputs (index l =
    // layer output), G0 / G1 [N][wp] adjoints
    auto Hs = [&](int bb, int l, int j) { return (T *)smem_raw + (size_t)bb * per + ((size_t)l * N + j) * wp; };
    auto Ts = [&](int bb, int l, int j) { return (T *)smem_raw + (size_t)bb * per + ((size_t)(L + l) * N + j) * wp; };
    auto Gb = [&](int bb, int q, int j) { return (T *)smem_raw + (size_t)bb * per + ((size_t)(2 * L + q) * N + j) * wp; };
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int q = tid; q < nwi * N; q += nt) {
        const int bb = q / N, j = q % N;
        const int64_t wi = wi0 + bb, w = wi / N;
        const int i = (int)(wi % N);
        const double *xw = x + w * 3 * N;
        T *p = Hs(bb, 0, j);
        for (int e = 0; e < wp; ++e) p[e] = T(0);
        if (j != i) {
            const double d0 = xw[3 * i] - xw[3 * j], d1 = xw[3 * i + 1] - xw[3 * j + 1], d2 = xw[3 * i + 2] - xw[3 * j + 2];
            p[0] = (T)d0; p[1] = (T)d1; p[2] = (T)d2;
            p[3] = (T)sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
    }
    __syncthreads();
    for (int l = 0; l + 1 < L; ++l) {
        const int dp = l == 0 ? 4 : s.w2;
        const T *W2 = Wsm + (P.W2[l] - P.W2[0]);
        const T *c2 = Wsm + (P.c2[l] - P.W2[0]);
        for (int q = tid; q < nwi * N * s.w2; q += nt) {
            const int o = q % s.w2, bj = q / s.w2, j = bj % N, bb = bj / N;
            const T *in = Hs(bb, l, j);
            T z = c2[o];
            for (int k = 0; k < dp; ++k) z += in[k] * W2[k * s.w2 + o];
            const T t = tanh(z);
            Ts(bb, l + 1, j)[o] = t;
            Hs(bb, l + 1, j)[o] = t + (l >= 1 ? in[o] : T(0));
        }
        __syncthreads();
    }
    const int nu = s.nu, nd = s.nd;
    auto mean_adj = [&](int bb, int l, int j, int o) -> T {
        const int dp = l == 0 ? 4 : s.w2;
        if (o >= dp) return T(0);
        const int spj = j < nu ? 0 : 1;
        const int n = spj == 0 ? nu : nd;
        return GGI[(int64_t)l * gg_layer_stride + (wi0 + bb) * ldg + spj * dp + o] / T(n);
    };
    // adjoint of the top pair state from the top layer's spin means (G0)
    for (int q = tid; q < nwi * N * wp; q += nt) {
        const int o = q % wp, bj = q / wp, j = bj % N, bb = bj / N;
        Gb(bb, 0, j)[o] = mean_adj(bb, L - 1, j, o);
    }
    __syncthreads();
    T *pp = PP + (int64_t)blockIdx.x * npp;
    for (int l = L - 1; l >= 1; --l) {
        // pair layer l - 1 maps h^{l-1} (width dp) to h^l (width w2)
        const int dp = l - 1 == 0 ? 4 : s.w2;
        const T *W2 = Wsm + (P.W2[l - 1] - P.W2[0]);
        // dz = G (1 - t^2) into G1
        for (int q = tid; q < nwi * N * s.w2; q += nt) {
            const int o = q % s.w2, bj = q / s.w2, j = bj % N, bb = bj / N;
            const T t = Ts(bb, l, j)[o];
            Gb(bb, 1, j)[o] = Gb(bb, 0, j)[o] * (T(1) - t * t);
        }
        __syncthreads();
        // dW2[k][o] = sum over the rows and pairs of h^{l-1}[k] dz[o], dc2[o] = sum dz[o]
        const int64_t wof = P.W2[l - 1] - P.W2[0], cof = P.c2[l - 1] - P.W2[0];
        for (int q = tid; q < (dp + 1) * s.w2; q += nt) {
            const int k = q / s.w2, o = q % s.w2;
            T acc = T(0);
            for (int bb = 0; bb < nwi; ++bb)
                for (int j = 0; j < N; ++j) acc += (k < dp ? Hs(bb, l - 1, j)[k] : T(1)) * Gb(bb, 1, j)[o];
            pp[k < dp ? wof + (int64_t)k * s.w2 + o : cof + o] = acc;
        }
        // adjoint of h^{l-1}: dz W2^T + residual + spin-mean part (into G0)
        __syncthreads();
        for (int q = tid; q < nwi * N * wp; q += nt) {
            const int k = q % wp, bj = q / wp, j = bj % N, bb = bj / N;
            T v = T(0);
            if (k < dp) {
                const T *dz = Gb(bb, 1, j);
                for (int o = 0; o < s.w2; ++o) v += dz[o] * W2[k * s.w2 + o];
                if (l - 1 >= 1) v += Gb(bb, 0, j)[k];
                v += mean_adj(bb, l - 1, j, k);
            }
            Gb(bb, 0, j)[k] = v;   // a thread reads only G1 and its own G0 entry
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// pair stream adjoint on the matrix cores (FP32 parameters): the quantities
// of k_pair_backward for WB (walker, electron) rows at once, each pair
// layer's three products as v_mfma_f32_16x16x4f32 over 16-row blocks of
// pairs:
//   forward recompute   z = h W2 + c2     (A: pair rows, B: packed W2^T)
//   activation adjoint  g = dz W2^T       (A: dz rows, B: W2 read from W2^T)
//   weight gradient     dW2 = h^T dz      (pairs are the reduction)
// LDS: the packed pair weights (matrix-core pair kernel layout), then slabs of
// round_up(WB N, 16) pair rows x (wc + 4) floats: features F, tanh outputs
// T_1 .. T_{L-1}, adjoint G, and D (the running activation during the
// recompute, dz afterwards).  The recompute repeats the forward kernel's
// operations in its order, and activations h^1 = T_1, h^l = T_l + h^{l-1}
// are rebuilt in the forward's order, so both equal the forward's values bit
// for bit.  Rows past the pairs held here get a zero adjoint.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pair_backward_mfma(Sys s, const double *x, const float *__restrict__ Wpk,
                                                            ParamLayout P, int64_t B, const float *GGI, int64_t ldg,
                                                            int64_t gg_layer_stride, int WB, float *PP, int64_t npp)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ float red[256];
    const int wc = round_up(s.w2, 16), RS = wc + 4, ncb = wc / 16;
    const int L = s.L, N = s.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, li = lane & 15;
    const int64_t wi0 = (int64_t)blockIdx.x * WB;
    const int nwi = B * N - wi0 < WB ? (int)(B * N - wi0) : WB;
    const int np = nwi * N;                           // pairs held here
    const int nal = round_up(WB * N, 16);             // rows per slab
    const int nblk = (np + 15) / 16;
    const int wtot = pair_mfma_woff(s, L - 1);
    float *Wsm = (float *)smem_raw;
    float *F = Wsm + wtot;
    auto Ts = [&](int l) { return F + (int64_t)l * nal * RS; };   // l = 1 .. L - 1
    float *G = F + (int64_t)L * nal * RS;
    float *D = G + (int64_t)nal * RS;
    for (int q = 4 * tid; q < wtot; q += 4 * blockDim.x) *(float4 *)(Wsm + q) = *(const float4 *)(Wpk + q);
    for (int q = 4 * tid; q < (L + 2) * nal * RS; q += 4 * blockDim.x)
        *(float4 *)(F + q) = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    for (int q = tid; q < np; q += blockDim.x) {
        const int bb = q / N, j = q % N;
        const int64_t wi = wi0 + bb, w = wi / N;
        const int i = (int)(wi % N);
        if (j == i) continue;
        const double *xw = x + w * 3 * N;
        const double d0 = xw[3 * i] - xw[3 * j], d1 = xw[3 * i + 1] - xw[3 * j + 1], d2 = xw[3 * i + 2] - xw[3 * j + 2];
        float *pf = F + (int64_t)q * RS, *pd = D + (int64_t)q * RS;
        pf[0] = pd[0] = (float)d0;
        pf[1] = pd[1] = (float)d1;
        pf[2] = pd[2] = (float)d2;
        pf[3] = pd[3] = (float)sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    __syncthreads();
    // forward recompute; D carries h^l
    for (int l = 0; l + 1 < L; ++l) {
        const int KP = pair_mfma_kp(s, l), KS = KP + 4;
        const float *Wl = Wsm + pair_mfma_woff(s, l);
        const float *bl = Wl + wc * KS;
        float *Tn = Ts(l + 1);
        for (int blk = wave; blk < nblk; blk += 4) {
            const int r0 = blk * 16;
            f32x4 acc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const float bv = cb < ncb ? bl[cb * 16 + li] : 0.f;
                acc[cb] = f32x4{bv, bv, bv, bv};
            }
            const float *arow = D + (int64_t)(r0 + li) * RS + 4 * g;
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
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (cb >= ncb) continue;
                const int64_t o = (int64_t)(r0 + 4 * g) * RS + cb * 16 + li;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float tv = tanhf(acc[cb][e]);
                    Tn[o + e * RS] = tv;
                    D[o + e * RS] = tv + (l >= 1 ? D[o + e * RS] : 0.f);
                }
            }
        }
        __syncthreads();
    }
    const int nu = s.nu, nd = s.nd;
    auto mean_adj = [&](int l, int p, int o) -> float {
        const int dp = layer_dp(s, l);
        if (o >= dp || p >= np) return 0.f;
        const int j = p % N, spj = j < nu ? 0 : 1;
        const int n = spj == 0 ? nu : nd;
        return GGI[(int64_t)l * gg_layer_stride + (wi0 + p / N) * ldg + spj * dp + o] / (float)n;
    };
    for (int q = tid; q < nal * wc; q += blockDim.x) {
        const int p = q / wc, o = q % wc;
        G[(int64_t)p * RS + o] = mean_adj(L - 1, p, o);
    }
    __syncthreads();
    float *pp = PP + (int64_t)blockIdx.x * npp;
    const int nparts = blockDim.x / wc;
    for (int l = L - 1; l >= 1; --l) {
        // pair layer l - 1 maps h^{l-1} (width dp) to h^l (width w2)
        const int dp = layer_dp(s, l - 1), KP = pair_mfma_kp(s, l - 1), KS = KP + 4;
        const float *Wl = Wsm + pair_mfma_woff(s, l - 1);
        const float *Tl = Ts(l);
        for (int q = tid; q < nal * wc; q += blockDim.x) {
            const int64_t e = (int64_t)(q / wc) * RS + q % wc;
            const float tv = Tl[e];
            D[e] = G[e] * (1.f - tv * tv);
        }
        __syncthreads();
        // dW2[k][o] = sum over pairs of h^{l-1}[k] dz[o]
        const int nkb = KP / 16;
        for (int ob = wave; ob < nkb * ncb; ob += 4) {
            const int kbk = ob / ncb, cb = ob % ncb;
            const int k = kbk * 16 + li, o = cb * 16 + li;
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int pb = 0; pb < nal; pb += 4) {
                const int64_t r = (int64_t)(pb + g) * RS;
                float h;
                if (l - 1 == 0) {
                    h = F[r + k];
                } else {
                    h = Ts(1)[r + k];
                    for (int m = 2; m <= l - 1; ++m) h = Ts(m)[r + k] + h;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(h, D[r + o], acc, 0, 0, 0);
            }
            const int64_t wof = P.W2[l - 1] - P.W2[0];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kk = kbk * 16 + 4 * g + e;
                if (kk < dp && o < s.w2) pp[wof + (int64_t)kk * s.w2 + o] = acc[e];
            }
        }
        // dc2[o] = sum over pairs of dz[o]: partial sums here, total below
        if (tid < nparts * wc) {
            const int o = tid % wc;
            float v = 0.f;
            for (int p = tid / wc; p < np; p += nparts) v += D[(int64_t)p * RS + o];
            red[tid] = v;
        }
        // adjoint of h^{l-1}: dz W2^T + residual + spin-mean part (into G)
        for (int blk = wave; blk < nblk; blk += 4) {
            const int r0 = blk * 16;
            const float *arow = D + (int64_t)(r0 + li) * RS + 4 * g;
            for (int kbk = 0; kbk < nkb; ++kbk) {
                f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
                for (int ob = 0; ob < wc; ob += 16) {
                    const float4 a4 = *(const float4 *)(arow + ob);
                    const float *wb = Wl + (ob + 4 * g) * KS + kbk * 16 + li;   // W2[k][o] = W2^T[o][k]
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, wb[0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, wb[KS], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, wb[2 * KS], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, wb[3 * KS], acc, 0, 0, 0);
                }
                const int k = kbk * 16 + li;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int p = r0 + 4 * g + e;
                    float *gp = G + (int64_t)p * RS + k;
                    float v = 0.f;
                    if (k < dp && p < np) v = acc[e] + (l - 1 >= 1 ? *gp : 0.f) + mean_adj(l - 1, p, k);
                    *gp = v;
                }
            }
        }
        __syncthreads();
        if (tid < s.w2) {
            float v = 0.f;
            for (int q = 0; q < nparts; ++q) v += red[q * wc + tid];
            pp[(P.c2[l - 1] - P.W2[0]) + tid] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// weight-gradient products C[a][b] = sum_r X[r][a] Y[r][b] (split over rows)
// partial[s][a][b] for row range s; X rows may be remapped by groups.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_tn_partial(const T *X, int64_t ldx, int NA, const T *Y, int64_t ldy, int NB,
                                                    int64_t R, int64_t per, int64_t stride, int64_t off,
                                                    int64_t rows_per_split, T *part)
{
    __shared__ T sx[16][64 + 1];
    __shared__ T sy[16][64 + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int a0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < R ? r0 + rows_per_split : R;
    T acc[4][4] = {};
    for (int64_t rb = r0; rb < r1; rb += 16) {
        for (int q = tid; q < 16 * 64; q += 256) {
            const int rr = q / 64, c = q % 64;
            const int64_t r = rb + rr;
            T vx = T(0), vy = T(0);
            if (r < r1) {
                const int64_t xr = per > 0 ? remap_row(r, per, stride, off) : r;
                if (a0 + c < NA) vx = X[xr * ldx + a0 + c];
                if (b0 + c < NB) vy = Y[r * ldy + b0 + c];
            }
            sx[rr][c] = vx;
            sy[rr][c] = vy;
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            T xa[4], yb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) { xa[u] = sx[rr][ty * 4 + u]; yb[u] = sy[rr][tx * 4 + u]; }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += xa[u] * yb[v];
        }
        __syncthreads();
    }
    T *p = part + (int64_t)blockIdx.z * NA * NB;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int a = a0 + ty * 4 + u;
        if (a >= NA) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int b = b0 + tx * 4 + v;
            if (b < NB) p[(int64_t)a * NB + b] = acc[u][v];
        }
    }
}

// FP32 on the matrix cores: the same 64 x 64 output tile, each wave a
// 32 x 32 quadrant (2 x 2 accumulators of v_mfma_f32_16x16x4f32, rows as the
// reduction dimension), rows staged 64 at a time; X^T and Y are both read
// straight from the row-major LDS tiles (lane: column lane & 15, row lane >> 4).
template <>
__global__ __launch_bounds__(256) void k_tn_partial<float>(const float *X, int64_t ldx, int NA, const float *Y,
                                                          int64_t ldy, int NB, int64_t R, int64_t per,
                                                          int64_t stride, int64_t off, int64_t rows_per_split,
                                                          float *part)
{
    constexpr int RC = 64, LS = 64 + 4;
    __shared__ float sx[RC][LS];
    __shared__ float sy[RC][LS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int a0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
    const int qa = (wave >> 1) * 32, qb = (wave & 1) * 32;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < R ? r0 + rows_per_split : R;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // a thread keeps column tid & 63 and rows tid / 64 + 4 u of a stage; all
    // of its loads are issued before the first store to LDS
    const int c = tid & 63, rq = tid >> 6;
    const bool cx = a0 + c < NA, cy = b0 + c < NB;
    for (int64_t rb = r0; rb < r1; rb += RC) {
        float vx[RC / 4], vy[RC / 4];
#pragma unroll
        for (int u = 0; u < RC / 4; ++u) {
            const int64_t r = rb + rq + 4 * u;
            vx[u] = 0.f;
            vy[u] = 0.f;
            if (r < r1) {
                const int64_t xr = per > 0 ? remap_row(r, per, stride, off) : r;
                if (cx) vx[u] = X[xr * ldx + a0 + c];
                if (cy) vy[u] = Y[r * ldy + b0 + c];
            }
        }
#pragma unroll
        for (int u = 0; u < RC / 4; ++u) {
            sx[rq + 4 * u][c] = vx[u];
            sy[rq + 4 * u][c] = vy[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < RC / 4; ++kk) {
            const int rr = 4 * kk + (lane >> 4);
            float fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) fa[i] = sx[rr][qa + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) fb[j] = sy[rr][qb + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator (i, j) element e: a = qa + 16 i + 4 (lane >> 4) + e, b = qb + 16 j + (lane & 15)
    float *p = part + (int64_t)blockIdx.z * NA * NB;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int a = a0 + qa + 16 * i + 4 * (lane >> 4) + e;
            if (a >= NA) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int b = b0 + qb + 16 * j + (lane & 15);
                if (b < NB) p[(int64_t)a * NB + b] = acc[i][j][e];
            }
        }
}

// acc[dst(a, b)] += sum_s part[s][a][b]; dst = off + a * lda_out + b
template <typename T>
__global__ void k_tn_reduce(const T *part, int S, int NA, int NB, double *acc, int64_t off, int64_t lda_out)
{
    const int64_t n = (int64_t)NA * NB;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int s = 0; s < S; ++s) v += (double)part[(int64_t)s * n + q];
        const int a = (int)(q / NB), b = (int)(q % NB);
        acc[off + (int64_t)a * lda_out + b] += v;
    }
}

// column sums: part[s][c] = sum over rows of split s of in[r][c]
template <typename T>
__global__ __launch_bounds__(256) void k_colsum_partial(const T *in, int64_t ld, int C, int64_t R,
                                                        int64_t rows_per_split, T *part)
{
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int ty = threadIdx.x >> 6;
    __shared__ double red[4][64];
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < R ? r0 + rows_per_split : R;
    double acc = 0.0;
    if (c < C) {
#pragma unroll 8
        for (int64_t r = r0 + ty; r < r1; r += 4) acc += (double)in[r * ld + c];
    }
    red[ty][threadIdx.x & 63] = acc;
    __syncthreads();
    if (ty == 0 && c < C) part[(int64_t)blockIdx.y * C + c] = (T)(red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// acc[map(c)] += sum_s part[s][c]; map (env_map = E > 0 partials per
// (column, nucleus)): envelope partials [col][m][E] go to pi [col][m] and
// Sigma [col][m][E - 1] (the nine entries, or the isotropic sigma);
// env_map = 0: acc[off + c]
template <typename T>
__global__ void k_colsum_reduce(const T *part, int S, int C, double *acc, int64_t off, int env_map, int64_t off2)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int s = 0; s < S; ++s) v += (double)part[(int64_t)s * C + c];
        if (!env_map) {
            acc[off + c] += v;
        } else {
            const int cm = c / env_map, e = c % env_map;      // cm = col * M + m
            if (e == 0) acc[off + cm] += v;
            else acc[off2 + (int64_t)cm * (env_map - 1) + (e - 1)] += v;
        }
    }
}

__global__ void k_zero_f64(double *p, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) p[q] = 0.0;
}

template <typename T>
__global__ void k_grad_out(const double *acc, int64_t n, T *grad)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) grad[q] = (T)acc[q];
}

// Wb[u][col] = w[u][col] for col < kn, 0 up to KNp (adjoint of the head);
// rounded to BF16 when the forward's head weights are (BF16-weight modes)
template <typename T>
__global__ void k_pack_head_bwd(const T *theta, int64_t woff, int w1, int kn, int KNp, bool round, T *Wb)
{
    const int64_t n = (int64_t)w1 * KNp;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int u = (int)(q / KNp), col = (int)(q % KNp);
        T v = col < kn ? theta[woff + (int64_t)u * kn + col] : T(0);
        if (round) v = (T)bf16_round((float)v);
        Wb[q] = v;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t det_backward_lds(int n) { return (size_t)2 * n * n * sizeof(double) + (size_t)n * sizeof(int) + 16; }

// ---------------------------------------------------------------------------
// pretraining loss of Eq. 5, (1/B) sum_w sum_{k,i,j} (Phi - Phi_target)^2
// over both spins: the adjoint of the orbital matrices and each walker's sum
// of squares, one thread per walker (entries in order, so the sums are
// reproducible); the loss reduction in one workgroup in a fixed order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pretrain_adjoint(const double *Phi, const double *target, int64_t B, int per,
                                                          double scale, double *GA, double *lsum)
{
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < B; w += (int64_t)gridDim.x * blockDim.x) {
        const double *p = Phi + w * per, *t = target + w * per;
        double *g = GA + w * per;
        double acc = 0.0;
        for (int q = 0; q < per; ++q) {
            const double d = p[q] - t[q];
            g[q] = scale * d;
            acc += d * d;
        }
        lsum[w] = acc;
    }
}

__global__ __launch_bounds__(1024) void k_pretrain_loss(const double *lsum, int64_t B, double *loss)
{
    __shared__ double red[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double acc = 0.0;
    for (int64_t p = tid; p < B; p += blockDim.x) acc += lsum[p] + lsum[B + p];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
        *loss = t / (double)B;
    }
}

void launch_pretrain_adjoint(const double *Phi, const double *target, int64_t B, int K, int n, double scale, double *GA,
                             double *lsum, hipStream_t st)
{
    hipLaunchKernelGGL(k_pretrain_adjoint, dim3(gridn(B)), dim3(256), 0, st, Phi, target, B, K * n * n, scale, GA,
                       lsum);
}

void launch_pretrain_loss(const double *lsum, int64_t B, double *loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_pretrain_loss, dim3(1), dim3(1024), 0, st, lsum, B, loss);
}

void launch_det_backward(const double *Phi, const double *DR, const double *coeff, int64_t B, int K, int n, int sp,
                         int nu, int nd, int rec, double *GA, hipStream_t st)
{
    const unsigned g = (unsigned)((B * K + 255) / 256);
    switch (n) {
#define FN_DBS(NS) \
    case NS: hipLaunchKernelGGL(k_det_backward_small<NS>, dim3(g), dim3(256), 0, st, Phi, DR, coeff, B, K, n, nu, nd, rec, GA); return;
        FN_DBS(1)
        FN_DBS(2)
        FN_DBS(3)
        FN_DBS(4)
        FN_DBS(5)
        FN_DBS(6)
        FN_DBS(7)
        FN_DBS(8)
#undef FN_DBS
    default: break;
    }
    hipLaunchKernelGGL(k_det_backward, dim3((unsigned)(B * K)), dim3(64), det_backward_lds(n), st, Phi, DR, coeff, B, K,
                       n, sp, nu, nd, rec, GA);
}

template <typename T>
void launch_env_backward(const Sys &s, const double *x, const T *theta, int64_t gof, int64_t piof, int64_t sigof,
                         int sp, const T *O, int64_t ldo, const double *GA, int64_t B, int KNp, T *Ga, T *EP,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_env_backward<T>, dim3(gridn(B * KNp, 128)), dim3(128), 0, st, s, x, theta, gof, piof, sigof,
                       sp, O, ldo, GA, B, KNp, Ga, EP);
}

template <typename T>
void launch_bwd_gz(const T *Gy, const T *Tt, int64_t B, int N, int w1, T *Gz, T *SGz, hipStream_t st)
{
    hipLaunchKernelGGL(k_bwd_gz<T>, dim3((unsigned)B), dim3(256), 0, st, Gy, Tt, N, w1, Gz, SGz);
}

template <typename T>
void launch_bwd_gh(const T *Gh, const T *Gy, const T *Gg, int64_t B, int N, int nu, int dh, int w1, int resid, T *Gout,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_bwd_gh<T>, dim3((unsigned)(B * N)), dim3(256), 0, st, Gh, Gy, Gg, N, nu, dh, w1, resid, Gout);
}

static size_t pair_backward_lds_wb(const Sys &s, size_t elem, int wb)
{
    const int wp = s.w2 > 4 ? s.w2 : 4;
    const ParamLayout P = make_layout(s);
    const size_t npw = s.L > 1 ? (size_t)(P.c2[s.L - 2] + s.w2 - P.W2[0]) : 0;
    return ((size_t)wb * (2 * (size_t)s.L + 2) * s.N * wp + npw) * elem;
}

size_t pair_backward_lds(const Sys &s, size_t elem) { return pair_backward_lds_wb(s, elem, 1); }

// (walker, electron) rows per workgroup: about 256 (pair, column) items,
// within 64 KiB of LDS
int pair_backward_wb(const Sys &s, size_t elem)
{
    const int items = s.N * s.w2;
    int wb = items >= 256 ? 1 : 256 / items;
    while (wb > 1 && pair_backward_lds_wb(s, elem, wb) > 64 * 1024) --wb;
    return wb;
}

// matrix-core adjoint: LDS of WB (walker, electron) rows; about 64 pairs per
// workgroup (one row block per wave) within 64 KiB
static size_t pair_backward_mfma_lds(const Sys &s, int wb)
{
    const int wc = round_up(s.w2, 16);
    const size_t nal = (size_t)round_up(wb * s.N, 16);
    return ((size_t)pair_mfma_woff(s, s.L - 1) + (size_t)(s.L + 2) * nal * (wc + 4)) * sizeof(float);
}

static int pair_backward_mfma_wb(const Sys &s)
{
    int wb = s.N >= 64 ? 1 : 64 / s.N;
    while (wb > 1 && pair_backward_mfma_lds(s, wb) > 64 * 1024) --wb;
    return wb;
}

template <typename T>
int64_t launch_pair_backward(const Sys &s, const double *x, const T *theta, const ParamLayout &P, int64_t B,
                             const T *GGI, int64_t ldg, int64_t gg_layer_stride, const float *wpair, T *PP,
                             int64_t npp, hipStream_t st)
{
    if constexpr (std::is_same<T, float>::value) {
        if (wpair && g_pair_mfma && s.w2 <= 64 && s.w2 % 4 == 0 && pair_backward_mfma_lds(s, 1) <= 64 * 1024) {
            const int wb = pair_backward_mfma_wb(s);
            const int64_t grid = (B * s.N + wb - 1) / wb;
            hipLaunchKernelGGL(k_pair_backward_mfma, dim3((unsigned)grid), dim3(256), pair_backward_mfma_lds(s, wb), st,
                               s, x, wpair, P, B, GGI, ldg, gg_layer_stride, wb, PP, npp);
            return grid;
        }
    }
    const int wb = pair_backward_wb(s, sizeof(T));
    const int64_t grid = (B * s.N + wb - 1) / wb;
    hipLaunchKernelGGL(k_pair_backward<T>, dim3((unsigned)grid), dim3(256), pair_backward_lds_wb(s, sizeof(T), wb), st,
                       s, x, theta, P, B, GGI, ldg, gg_layer_stride, wb, PP, npp);
    return grid;
}

int tn_splits(int64_t R)
{
    int64_t s = R / 512;
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    return (int)s;
}

template <typename T>
void launch_tn(const T *X, int64_t ldx, int NA, const T *Y, int64_t ldy, int NB, int64_t R, int64_t per,
               int64_t stride, int64_t off, T *part, double *acc, int64_t acc_off, int64_t lda_out, hipStream_t st)
{
    if (R <= 0 || NA <= 0 || NB <= 0) return;
    const int S = tn_splits(R);
    const int64_t rps = (R + S - 1) / S;
    dim3 g((unsigned)((NA + 63) / 64), (unsigned)((NB + 63) / 64), (unsigned)S);
    hipLaunchKernelGGL(k_tn_partial<T>, g, dim3(256), 0, st, X, ldx, NA, Y, ldy, NB, R, per, stride, off, rps, part);
    hipLaunchKernelGGL(k_tn_reduce<T>, dim3(gridn((int64_t)NA * NB)), dim3(256), 0, st, part, S, NA, NB, acc, acc_off,
                       lda_out);
}

template <typename T>
void launch_colsum(const T *in, int64_t ld, int C, int64_t R, T *part, double *acc, int64_t off, int env_map,
                   int64_t off2, hipStream_t st)
{
    if (R <= 0 || C <= 0) return;
    const int S = tn_splits(R);
    const int64_t rps = (R + S - 1) / S;
    hipLaunchKernelGGL(k_colsum_partial<T>, dim3((unsigned)((C + 63) / 64), (unsigned)S), dim3(256), 0, st, in, ld, C, R,
                       rps, part);
    hipLaunchKernelGGL(k_colsum_reduce<T>, dim3(gridn(C)), dim3(256), 0, st, part, S, C, acc, off, env_map, off2);
}

int max_splits() { return 64; }

void launch_zero_f64(double *p, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_f64, dim3(gridn(n)), dim3(256), 0, st, p, n);
}

template <typename T>
void launch_grad_out(const double *acc, int64_t n, T *grad, hipStream_t st)
{
    hipLaunchKernelGGL(k_grad_out<T>, dim3(gridn(n)), dim3(256), 0, st, acc, n, grad);
}

template <typename T>
void launch_pack_head_bwd(const T *theta, int64_t woff, int w1, int kn, int KNp, bool round, T *Wb, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_head_bwd<T>, dim3(gridn((int64_t)w1 * KNp)), dim3(256), 0, st, theta, woff, w1, kn, KNp,
                       round, Wb);
}

#define FN_BWD_INST(T)                                                                                               \
    template void launch_env_backward<T>(const Sys &, const double *, const T *, int64_t, int64_t, int64_t, int,       \
                                         const T *, int64_t, const double *, int64_t, int, T *, T *, hipStream_t);    \
    template void launch_bwd_gz<T>(const T *, const T *, int64_t, int, int, T *, T *, hipStream_t);                   \
    template void launch_bwd_gh<T>(const T *, const T *, const T *, int64_t, int, int, int, int, int, T *,           \
                                   hipStream_t);                                                                      \
    template int64_t launch_pair_backward<T>(const Sys &, const double *, const T *, const ParamLayout &, int64_t,    \
                                             const T *, int64_t, int64_t, const float *, T *, int64_t, hipStream_t);  \
    template void launch_tn<T>(const T *, int64_t, int, const T *, int64_t, int, int64_t, int64_t, int64_t, int64_t,  \
                               T *, double *, int64_t, int64_t, hipStream_t);                                         \
    template void launch_colsum<T>(const T *, int64_t, int, int64_t, T *, double *, int64_t, int, int64_t,           \
                                   hipStream_t);                                                                      \
    template void launch_grad_out<T>(const double *, int64_t, T *, hipStream_t);                                      \
    template void launch_pack_head_bwd<T>(const T *, int64_t, int, int, int, bool, T *, hipStream_t);

FN_BWD_INST(float)
FN_BWD_INST(double)

}  // namespace fn
