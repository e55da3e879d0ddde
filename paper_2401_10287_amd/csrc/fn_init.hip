// fn_init.hip -- electron counts and initial walkers (paper: Ionic Charge
// Initialization section, Algorithm 1; Electron Sampler section).
//
// fn_ionic_electron_counts: Algorithm 1 on the host.  Starting from the
// neutral counts (the atomic numbers) and the ion's charge t, each step
// takes one electron from the nucleus of largest partial charge (t > 0) or
// gives one to the nucleus of smallest partial charge (t < 0), moves t one
// step towards zero, and shifts that nucleus's partial charge by one in the
// direction that makes it less likely to be picked again (as the algorithm
// states).  Ties go to the lowest index.
//
// fn_init_walkers: electrons placed about their nuclei with Gaussian
// offsets, x = R[site(i)] + scale z, z from the sampler's generator at
// counter step 0xFFFFFFFF.
#include <math.h>

#include "fn_internal.h"

namespace fn {
namespace {

// electron i's nucleus position, 3 N doubles passed by value
struct SiteXYZ {
    double v[3 * FN_MAX_ELEC];
};

// one (walker, deviate pair) per item: coordinates q = 2 d and 2 d + 1
__global__ __launch_bounds__(256) void k_init_walkers(SiteXYZ sites, int64_t B, int n3, double scale, uint32_t key0,
                                                      uint32_t key1, uint32_t stream_id, double *x)
{
#pragma clang fp contract(off)
    const int nd = (n3 + 1) / 2;
    const int64_t total = B * nd;
    for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = it / nd;
        const int d = (int)(it - w * nd);
        uint32_t c[4] = {(uint32_t)d, (uint32_t)w, 0xFFFFFFFFu, stream_id};
        philox4x32_10(c, key0, key1);
        const double u1 = word_pair_to_unit(c[0], c[1]), u2 = word_pair_to_unit(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1)), ang = 2.0 * M_PI * u2;
        const int q = 2 * d;
        const double s0 = scale * (rad * cos(ang));
        x[w * n3 + q] = sites.v[q] + s0;
        if (q + 1 < n3) {
            const double s1 = scale * (rad * sin(ang));
            x[w * n3 + q + 1] = sites.v[q + 1] + s1;
        }
    }
}

}  // namespace
}  // namespace fn

using namespace fn;

extern "C" {

fn_status fn_ionic_electron_counts(int32_t n_nuc, const double *partial_charge, const int32_t *atomic_number,
                                   int32_t ion_charge, int32_t *electrons)
{
    if (n_nuc < 1 || n_nuc > FN_MAX_NUC) return api_fail(FN_EINVAL, "n_nuc out of range 1..32");
    if (!partial_charge || !atomic_number || !electrons) return api_fail(FN_EINVAL, "NULL argument");
    double charge[FN_MAX_NUC];
    int32_t e[FN_MAX_NUC];
    int64_t total = 0;
    for (int m = 0; m < n_nuc; ++m) {
        if (!isfinite(partial_charge[m])) return api_fail(FN_EINVAL, "non-finite partial charge");
        if (atomic_number[m] < 0) return api_fail(FN_EINVAL, "negative atomic number");
        charge[m] = partial_charge[m];
        e[m] = atomic_number[m];
        total += e[m];
    }
    if ((int64_t)ion_charge > total) return api_fail(FN_EINVAL, "ion charge exceeds the electron count");
    if ((int64_t)total - ion_charge > FN_MAX_ELEC) return api_fail(FN_EUNSUPPORTED, "more than 32 electrons");
    int32_t t = ion_charge;
    while (t != 0) {
        int idx = 0;
        if (t < 0) {
            for (int m = 1; m < n_nuc; ++m)
                if (charge[m] < charge[idx]) idx = m;
            e[idx] += 1;
            t += 1;
            charge[idx] += 1.0;
        } else {
            for (int m = 1; m < n_nuc; ++m)
                if (charge[m] > charge[idx]) idx = m;
            if (e[idx] == 0) return api_fail(FN_EINVAL, "the policy would take an electron from an empty nucleus");
            e[idx] -= 1;
            t -= 1;
            charge[idx] -= 1.0;
        }
    }
    for (int m = 0; m < n_nuc; ++m) electrons[m] = e[m];
    return FN_OK;
}

fn_status fn_init_walkers(const fn_config *cfg, const int32_t *site, double scale, uint64_t seed, uint32_t stream_id,
                          int64_t B, double *x, void *stream)
{
    if (!cfg || !site) return api_fail(FN_EINVAL, "cfg or site is NULL");
    if (cfg->n_nuc < 1 || cfg->n_nuc > FN_MAX_NUC || !cfg->nuc_xyz) return api_fail(FN_EINVAL, "bad nuclei");
    const int N = cfg->n_up + cfg->n_down;
    if (cfg->n_up < 0 || cfg->n_down < 0 || N < 1 || N > FN_MAX_ELEC) return api_fail(FN_EINVAL, "bad electron count");
    if (B < 0) return api_fail(FN_EINVAL, "B < 0");
    if (B > 0 && !x) return api_fail(FN_EINVAL, "x is NULL");
    if (!(scale >= 0.0) || !isfinite(scale)) return api_fail(FN_EINVAL, "scale must be finite and >= 0");
    SiteXYZ sites{};
    for (int i = 0; i < N; ++i) {
        if (site[i] < 0 || site[i] >= cfg->n_nuc) return api_fail(FN_EINVAL, "site index out of range");
        for (int a = 0; a < 3; ++a) sites.v[3 * i + a] = cfg->nuc_xyz[3 * site[i] + a];
    }
    if (B == 0) return FN_OK;
    const int n3 = 3 * N;
    const int64_t total = B * ((n3 + 1) / 2);
    int64_t g = (total + 255) / 256;
    if (g > 1 << 20) g = 1 << 20;
    hipLaunchKernelGGL(k_init_walkers, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream, sites, B, n3, scale,
                       (uint32_t)seed, (uint32_t)(seed >> 32), stream_id, x);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return api_fail(FN_EHIP, hipGetErrorString(err));
    return FN_OK;
}

}  // extern "C"
