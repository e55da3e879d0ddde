// fn_mc.hip -- Metropolis-Hastings walker update (Electron Sampler section
// of the paper) and the batch energy statistics of Eq. 1 and Eq. 6.
//
// Proposal: every electron of a walker moves by sigma z, z ~ N(0, 1); the
// move is kept iff log|psi'| is finite and log u <= 2 (log|psi'| - log|psi|)
// (decided in the combine kernel of the proposal's value pass, fn_net.hip).
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// with key (seed low, seed high) and counter (d, walker, step, stream_id);
// normal deviates by the Box-Muller transform (1958).
#include "fn_internal.h"
#include "fn_kernels.h"

namespace fn {

// Deviate pair d of walker w (d < ceil(3N/2): coordinates 2 d and 2 d + 1,
// x' = x + sigma z rounded as a product and then a sum, no fused
// multiply-add), or its accept uniform (d == ceil(3N/2)).  The generator
// counter takes the walker's index within its own job, wl.
__device__ inline void propose_item(const double *x, int64_t w, int64_t wl, int d, int n3, double sigma, uint32_t k0,
                                    uint32_t k1, uint32_t step, uint32_t stream_id, const double *z_ext,
                                    const double *u_ext, double *xp, double *u)
{
#pragma clang fp contract(off)
    const int D = (n3 + 1) / 2;
    if (d == D) {
        if (u_ext) {
            u[w] = u_ext[w];
        } else {
            uint32_t c[4] = {0xFFFFFFFFu, (uint32_t)wl, step, stream_id};
            philox4x32_10(c, k0, k1);
            u[w] = word_pair_to_unit(c[0], c[1]);
        }
        return;
    }
    double z0, z1;
    if (z_ext) {
        z0 = z_ext[w * n3 + 2 * d];
        z1 = 2 * d + 1 < n3 ? z_ext[w * n3 + 2 * d + 1] : 0.0;
    } else {
        uint32_t c[4] = {(uint32_t)d, (uint32_t)wl, step, stream_id};
        philox4x32_10(c, k0, k1);
        const double u1 = word_pair_to_unit(c[0], c[1]), u2 = word_pair_to_unit(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 2.0 * M_PI * u2;
        z0 = rad * cos(ang);
        z1 = rad * sin(ang);
    }
    const double s0 = sigma * z0;
    xp[w * n3 + 2 * d] = x[w * n3 + 2 * d] + s0;
    if (2 * d + 1 < n3) {
        const double s1 = sigma * z1;
        xp[w * n3 + 2 * d + 1] = x[w * n3 + 2 * d + 1] + s1;
    }
}

// one thread per (walker, d), d = 0 .. ceil(3N/2)
__global__ void k_propose(const double *x, int64_t B, int n3, double sigma, uint32_t k0, uint32_t k1, uint32_t step,
                          uint32_t stream_id, const double *z_ext, const double *u_ext, double *xp, double *u)
{
    const int D = (n3 + 1) / 2;
    const int64_t total = B * (D + 1);
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total; id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = id / (D + 1);
        propose_item(x, w, w, (int)(id % (D + 1)), n3, sigma, k0, k1, step, stream_id, z_ext, u_ext, xp, u);
    }
}

// the same over the walkers of several jobs: job q owns walkers
// [w0[q], w0[q + 1]) and its own key, step counter and stream id
__global__ void k_propose_group(const double *x, int64_t B, int n3, double sigma, GroupTable g, double *xp, double *u)
{
    const int D = (n3 + 1) / 2;
    const int64_t total = B * (D + 1);
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total; id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = id / (D + 1);
        int lo = 0, hi = g.n - 1;                    // last job with w0 <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g.w0[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        propose_item(x, w, w - g.w0[lo], (int)(id % (D + 1)), n3, sigma, g.k0[lo], g.k1[lo], g.step[lo],
                     g.stream[lo], nullptr, nullptr, xp, u);
    }
}

// FP64 batch statistics of the local energy (Eq. 1): mean, variance (1/B),
// standard error; optional Eq. 6 coefficients c_p = 2 (E_p - mean) / B.
__global__ __launch_bounds__(1024) void k_energy_stats(const double *e, int64_t B, double *stats, double *coeff)
{
    __shared__ double red[32];
    __shared__ double s_mean;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double acc = 0.0;
    for (int64_t p = tid; p < B; p += blockDim.x) acc += e[p];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
        s_mean = t / (double)B;
    }
    __syncthreads();
    const double mean = s_mean;
    acc = 0.0;
    for (int64_t p = tid; p < B; p += blockDim.x) {
        const double d = e[p] - mean;
        acc += d * d;
        if (coeff) coeff[p] = 2.0 * d / (double)B;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __syncthreads();
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
        const double var = t / (double)B;
        if (stats) { stats[0] = mean; stats[1] = var; stats[2] = sqrt(var / (double)B); }
    }
}

static unsigned grid_of(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 1 << 20) g = 1 << 20;
    return (unsigned)(g < 1 ? 1 : g);
}

void launch_propose(const double *x, int64_t B, int n3, double sigma, uint64_t seed, uint64_t step, uint32_t stream_id,
                    const double *z_ext, const double *u_ext, double *xp, double *u, hipStream_t st)
{
    const int64_t total = B * ((n3 + 1) / 2 + 1);
    hipLaunchKernelGGL(k_propose, dim3(grid_of(total)), dim3(256), 0, st, x, B, n3, sigma, (uint32_t)seed,
                       (uint32_t)(seed >> 32), (uint32_t)step, stream_id, z_ext, u_ext, xp, u);
}

void launch_propose_group(const double *x, int64_t B, int n3, double sigma, const GroupTable &g, double *xp,
                          double *u, hipStream_t st)
{
    const int64_t total = B * ((n3 + 1) / 2 + 1);
    hipLaunchKernelGGL(k_propose_group, dim3(grid_of(total)), dim3(256), 0, st, x, B, n3, sigma, g, xp, u);
}

void launch_energy_stats(const double *e_loc, int64_t B, double *stats, double *coeff, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy_stats, dim3(1), dim3(1024), 0, st, e_loc, B, stats, coeff);
}

}  // namespace fn
