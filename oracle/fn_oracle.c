/*
 * fn_oracle.c -- plain FP64 CPU oracle for the FermiNet VMC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP path is checked against.  It is loaded only by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark; the product path
 * never links, imports or calls it.  It shares no code, header, table or
 * constant with the GPU library: the only thing both sides agree on is the
 * flat parameter layout and the random-number specification, each written
 * out here again from its definition.
 *
 * What it computes (paper: "Open-Source Fermionic Neural Networks with Ionic
 * Charge Initialization", Introduction and Implementation sections):
 *   - log|psi| of the FermiNet ansatz (Implementation / FermiNet Model, the
 *     one- and two-electron feature streams, the envelope of Eq. 4 and the
 *     Slater determinants built from envelope x orbital);
 *   - the local energy of Eq. 2, with the kinetic term of Eq. 3 read as
 *     -1/2 * sum over all 3N Cartesian coordinates of
 *     ((d log|psi|/dx_c)^2 + d^2 log|psi|/dx_c^2);
 *   - the Metropolis-Hastings walker update of the Electron Sampler section
 *     (Gaussian proposal, accept iff log u <= 2 log|psi'| - 2 log|psi|);
 *   - directional derivatives d log|psi| / d theta used to assemble the
 *     training gradient of Eq. 6.
 *
 * Method: every scalar is a hyper-dual number a + b e1 + c e2 + d e1 e2
 * (Fike & Alonso, 2011).  Seeding coordinate x_c with e1 + e2 gives the exact
 * first derivative in b and the exact second derivative in d, with no
 * truncation error, so the kinetic term is the plain definition evaluated
 * one coordinate at a time.  Seeding a parameter direction v in b alone
 * gives the exact directional derivative of log|psi| along v.
 *
 * Network reading used where the paper is silent (tanh activations,
 * residuals when in-width equals out-width, L one-electron layers and L-1
 * two-electron layers, mean-field inputs [h_i, g_up, g_dn, g_i_up, g_i_dn],
 * anisotropic envelope exp(-|Sigma (r_j - R_m)|) with a 3x3 Sigma per
 * orbital and nucleus, or the isotropic special case Sigma = sigma I with
 * one scalar sigma per orbital and nucleus, psi = sum_k det A_k_up *
 * det A_k_dn, self pairs included with |r_ii| := 0).
 *
 * Parameter layout (flat, FP64 here):
 *   for l = 0..L-1 : V_l [d_in][w1]  (d_in rows ordered h_i, g_up, g_dn,
 *                                     g_i_up, g_i_dn), b_l [w1]
 *   for l = 0..L-2 : W2_l [d_p][w2], c2_l [w2]
 *   for spin s = up, dn with n_s > 0:
 *                    w_s [w1][K n_s] (column k n_s + i), g_s [K n_s],
 *                    pi_s [K n_s][M], Sig_s [K n_s][M][3][3]
 *                    (isotropic envelope: sigma_s [K n_s][M])
 *   with d_h = 4M, d_p = 4 at layer 0 and d_h = w1, d_p = w2 after,
 *   d_in = 3 d_h + 2 d_p.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------ */
/* hyper-dual arithmetic                                               */
/* ------------------------------------------------------------------ */
typedef struct { double a, b, c, d; } hd;

static hd hconst(double a) { hd r = {a, 0.0, 0.0, 0.0}; return r; }
static hd hadd(hd x, hd y) { hd r = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; return r; }
static hd hsub(hd x, hd y) { hd r = {x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d}; return r; }
static hd hscale(hd x, double s) { hd r = {x.a * s, x.b * s, x.c * s, x.d * s}; return r; }
static hd hmul(hd x, hd y)
{
    hd r;
    r.a = x.a * y.a;
    r.b = x.a * y.b + x.b * y.a;
    r.c = x.a * y.c + x.c * y.a;
    r.d = x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a;
    return r;
}
/* f(x) for a hyper-dual x, given f, f', f'' at the real part */
static hd hchain(hd x, double f0, double f1, double f2)
{
    hd r;
    r.a = f0;
    r.b = f1 * x.b;
    r.c = f1 * x.c;
    r.d = f1 * x.d + f2 * x.b * x.c;
    return r;
}
static hd htanh(hd x) { double t = tanh(x.a); return hchain(x, t, 1.0 - t * t, -2.0 * t * (1.0 - t * t)); }
static hd hexp(hd x) { double e = exp(x.a); return hchain(x, e, e, e); }
static hd hsqrt(hd x) { double s = sqrt(x.a); return hchain(x, s, 0.5 / s, -0.25 / (s * x.a)); }
static hd hrecip(hd x) { double i = 1.0 / x.a; return hchain(x, i, -i * i, 2.0 * i * i * i); }
static hd hlogabs(hd x) { double i = 1.0 / x.a; return hchain(x, log(fabs(x.a)), i, -i * i); }

/* ------------------------------------------------------------------ */
/* configuration and parameter layout                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_nuc;
    const double *nuc_xyz; /* [M][3] */
    const double *nuc_z;   /* [M]    */
    int32_t n_up, n_dn, n_layers, w1, w2, n_det;
    int32_t envelope;      /* 0: Sigma 3x3 per orbital and nucleus; 1: Sigma = sigma I */
} orc_cfg;

typedef struct {
    int64_t V[64], b[64], W2[64], c2[64];
    int64_t w[2], g[2], pi[2], sig[2];
    int64_t total;
} orc_layout;

static int din_of(const orc_cfg *c, int l) { return l == 0 ? 3 * 4 * c->n_nuc + 2 * 4 : 3 * c->w1 + 2 * c->w2; }
static int dh_of(const orc_cfg *c, int l) { return l == 0 ? 4 * c->n_nuc : c->w1; }
static int dp_of(const orc_cfg *c, int l) { return l == 0 ? 4 : c->w2; }

static void make_layout(const orc_cfg *c, orc_layout *L)
{
    int64_t o = 0;
    for (int l = 0; l < c->n_layers; ++l) {
        L->V[l] = o; o += (int64_t)din_of(c, l) * c->w1;
        L->b[l] = o; o += c->w1;
    }
    for (int l = 0; l + 1 < c->n_layers; ++l) {
        L->W2[l] = o; o += (int64_t)dp_of(c, l) * c->w2;
        L->c2[l] = o; o += c->w2;
    }
    for (int s = 0; s < 2; ++s) {
        int ns = s == 0 ? c->n_up : c->n_dn;
        if (ns == 0) { L->w[s] = L->g[s] = L->pi[s] = L->sig[s] = -1; continue; }
        int kn = c->n_det * ns;
        L->w[s] = o; o += (int64_t)c->w1 * kn;
        L->g[s] = o; o += kn;
        L->pi[s] = o; o += (int64_t)kn * c->n_nuc;
        L->sig[s] = o; o += (int64_t)kn * c->n_nuc * (c->envelope ? 1 : 9);
    }
    L->total = o;
}

int64_t orc_param_count(const orc_cfg *c)
{
    orc_layout L;
    make_layout(c, &L);
    return L.total;
}

/* parameter i as a hyper-dual number: value theta[i], e1 part dir[i] */
static hd P(const double *th, const double *dir, int64_t i)
{
    hd r = {th[i], dir ? dir[i] : 0.0, 0.0, 0.0};
    return r;
}

/* ------------------------------------------------------------------ */
/* slogdet by LU with partial pivoting (pivot on the real part, first   */
/* row with the largest magnitude wins a tie)                          */
/* ------------------------------------------------------------------ */
static void lu_slogdet(int n, hd *A /* [n][n], destroyed */, int *sign, hd *logabs)
{
    int s = 1;
    hd acc = hconst(0.0);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k].a);
        for (int r = k + 1; r < n; ++r) {
            double v = fabs(A[r * n + k].a);
            if (v > best) { best = v; p = r; }
        }
        if (best == 0.0) {
            *sign = 0;
            logabs->a = -INFINITY; logabs->b = logabs->c = logabs->d = NAN;
            return;
        }
        if (p != k) {
            for (int cc = 0; cc < n; ++cc) { hd t = A[k * n + cc]; A[k * n + cc] = A[p * n + cc]; A[p * n + cc] = t; }
            s = -s;
        }
        hd piv = A[k * n + k];
        if (piv.a < 0) s = -s;
        acc = hadd(acc, hlogabs(piv));
        hd ipiv = hrecip(piv);
        for (int r = k + 1; r < n; ++r) {
            hd f = hmul(A[r * n + k], ipiv);
            for (int cc = k + 1; cc < n; ++cc) A[r * n + cc] = hsub(A[r * n + cc], hmul(f, A[k * n + cc]));
        }
    }
    *sign = s;
    *logabs = acc;
}

/* plain-double entry for checking the LU against a library slogdet */
void orc_slogdet(int32_t n, int64_t count, const double *A /*[count][n][n]*/, double *sign, double *logabs)
{
    hd *M = (hd *)malloc(sizeof(hd) * (size_t)(n > 0 ? n * n : 1));
    for (int64_t t = 0; t < count; ++t) {
        for (int i = 0; i < n * n; ++i) M[i] = hconst(A[t * n * n + i]);
        int s; hd l;
        if (n == 0) { s = 1; l = hconst(0.0); } else lu_slogdet(n, M, &s, &l);
        sign[t] = s;
        logabs[t] = l.a;
    }
    free(M);
}

/* ------------------------------------------------------------------ */
/* one walker: log|psi| and sign                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    hd *h1, *h1n, *h2, *h2n, *f, *gu, *gd, *giu, *gid, *A;
    hd *hL_out;     /* optional copy of the final one-electron stream          */
    double *mats;   /* optional copy of the orbital matrices [2][K][nmax][nmax] */
    double *mats_b; /* optional: their derivative along the parameter direction */
} scratch;

static scratch scratch_alloc(const orc_cfg *c)
{
    int N = c->n_up + c->n_dn;
    int dmax = 4 * c->n_nuc > c->w1 ? 4 * c->n_nuc : c->w1;
    int pmax = c->w2 > 4 ? c->w2 : 4;
    int nmax = c->n_up > c->n_dn ? c->n_up : c->n_dn;
    int dinmax = din_of(c, 0) > din_of(c, 1) ? din_of(c, 0) : din_of(c, 1);
    scratch s;
    s.h1 = (hd *)calloc((size_t)N * dmax, sizeof(hd));
    s.h1n = (hd *)calloc((size_t)N * dmax, sizeof(hd));
    s.h2 = (hd *)calloc((size_t)N * N * pmax, sizeof(hd));
    s.h2n = (hd *)calloc((size_t)N * N * pmax, sizeof(hd));
    s.f = (hd *)calloc((size_t)dinmax, sizeof(hd));
    s.gu = (hd *)calloc((size_t)dmax, sizeof(hd));
    s.gd = (hd *)calloc((size_t)dmax, sizeof(hd));
    s.giu = (hd *)calloc((size_t)pmax, sizeof(hd));
    s.gid = (hd *)calloc((size_t)pmax, sizeof(hd));
    s.A = (hd *)calloc((size_t)(nmax * nmax > 0 ? nmax * nmax : 1), sizeof(hd));
    s.hL_out = NULL;
    s.mats = NULL;
    s.mats_b = NULL;
    return s;
}

static void scratch_free(scratch *s)
{
    free(s->h1); free(s->h1n); free(s->h2); free(s->h2n); free(s->f);
    free(s->gu); free(s->gd); free(s->giu); free(s->gid); free(s->A);
}

/* the distance |v| of a 3-vector; callers never pass the zero vector */
static hd hnorm3(hd x, hd y, hd z) { return hsqrt(hadd(hadd(hmul(x, x), hmul(y, y)), hmul(z, z))); }

/*
 * x: [N][3] hyper-dual coordinates.  Writes log|psi| (hyper-dual) and the
 * sign of psi; optionally the per-(spin, det) slogdets dets[2][K][2].
 */
static void eval_walker(const orc_cfg *c, const orc_layout *Ly, const double *th, const double *dir,
                        const hd *x, scratch *S, hd *logpsi, int *sign, double *dets_out)
{
    const int M = c->n_nuc, N = c->n_up + c->n_dn, nu = c->n_up, nd = c->n_dn;
    const int w1 = c->w1, w2 = c->w2, K = c->n_det, Lyr = c->n_layers;
    const int dmax = 4 * M > w1 ? 4 * M : w1;
    const int pmax = w2 > 4 ? w2 : 4;
#define H1(i, k) S->h1[(i) * dmax + (k)]
#define H1N(i, k) S->h1n[(i) * dmax + (k)]
#define H2(i, j, k) S->h2[((i) * N + (j)) * pmax + (k)]
#define H2N(i, j, k) S->h2n[((i) * N + (j)) * pmax + (k)]

    /* input features: electron-nucleus [r_i - R_m, |r_i - R_m|] */
    for (int i = 0; i < N; ++i)
        for (int m = 0; m < M; ++m) {
            hd d0 = hsub(x[3 * i + 0], hconst(c->nuc_xyz[3 * m + 0]));
            hd d1 = hsub(x[3 * i + 1], hconst(c->nuc_xyz[3 * m + 1]));
            hd d2 = hsub(x[3 * i + 2], hconst(c->nuc_xyz[3 * m + 2]));
            H1(i, 4 * m + 0) = d0;
            H1(i, 4 * m + 1) = d1;
            H1(i, 4 * m + 2) = d2;
            H1(i, 4 * m + 3) = hnorm3(d0, d1, d2);
        }
    /* electron-electron [r_i - r_j, |r_i - r_j|]; the self pair is zero */
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            if (i == j) { for (int k = 0; k < 4; ++k) H2(i, j, k) = hconst(0.0); continue; }
            hd d0 = hsub(x[3 * i + 0], x[3 * j + 0]);
            hd d1 = hsub(x[3 * i + 1], x[3 * j + 1]);
            hd d2 = hsub(x[3 * i + 2], x[3 * j + 2]);
            H2(i, j, 0) = d0; H2(i, j, 1) = d1; H2(i, j, 2) = d2;
            H2(i, j, 3) = hnorm3(d0, d1, d2);
        }

    for (int l = 0; l < Lyr; ++l) {
        const int dh = dh_of(c, l), dp = dp_of(c, l), din = din_of(c, l);
        /* spin means of the one-electron stream */
        for (int k = 0; k < dh; ++k) {
            hd su = hconst(0.0), sd = hconst(0.0);
            for (int j = 0; j < nu; ++j) su = hadd(su, H1(j, k));
            for (int j = nu; j < N; ++j) sd = hadd(sd, H1(j, k));
            S->gu[k] = nu ? hscale(su, 1.0 / nu) : hconst(0.0);
            S->gd[k] = nd ? hscale(sd, 1.0 / nd) : hconst(0.0);
        }
        for (int i = 0; i < N; ++i) {
            /* spin means of the pair stream seen from electron i */
            for (int k = 0; k < dp; ++k) {
                hd su = hconst(0.0), sd = hconst(0.0);
                for (int j = 0; j < nu; ++j) su = hadd(su, H2(i, j, k));
                for (int j = nu; j < N; ++j) sd = hadd(sd, H2(i, j, k));
                S->giu[k] = nu ? hscale(su, 1.0 / nu) : hconst(0.0);
                S->gid[k] = nd ? hscale(sd, 1.0 / nd) : hconst(0.0);
            }
            int o = 0;
            for (int k = 0; k < dh; ++k) S->f[o++] = H1(i, k);
            for (int k = 0; k < dh; ++k) S->f[o++] = S->gu[k];
            for (int k = 0; k < dh; ++k) S->f[o++] = S->gd[k];
            for (int k = 0; k < dp; ++k) S->f[o++] = S->giu[k];
            for (int k = 0; k < dp; ++k) S->f[o++] = S->gid[k];
            for (int u = 0; u < w1; ++u) {
                hd acc = P(th, dir, Ly->b[l] + u);
                for (int k = 0; k < din; ++k) acc = hadd(acc, hmul(S->f[k], P(th, dir, Ly->V[l] + (int64_t)k * w1 + u)));
                hd y = htanh(acc);
                if (l >= 1) y = hadd(y, H1(i, u));
                H1N(i, u) = y;
            }
        }
        if (l + 1 < Lyr) {
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j)
                    for (int u = 0; u < w2; ++u) {
                        hd acc = P(th, dir, Ly->c2[l] + u);
                        for (int k = 0; k < dp; ++k)
                            acc = hadd(acc, hmul(H2(i, j, k), P(th, dir, Ly->W2[l] + (int64_t)k * w2 + u)));
                        hd y = htanh(acc);
                        if (l >= 1) y = hadd(y, H2(i, j, u));
                        H2N(i, j, u) = y;
                    }
            hd *t = S->h2; S->h2 = S->h2n; S->h2n = t;
        }
        hd *t = S->h1; S->h1 = S->h1n; S->h1n = t;
    }
    if (S->hL_out)
        for (int i = 0; i < N; ++i)
            for (int u = 0; u < w1; ++u) S->hL_out[i * w1 + u] = H1(i, u);

    /* orbitals x envelope, determinants, sum over determinants */
    int sk[64];
    hd lk[64];
    for (int k = 0; k < K; ++k) { sk[k] = 1; lk[k] = hconst(0.0); }
    for (int s = 0; s < 2; ++s) {
        const int ns = s == 0 ? nu : nd, j0 = s == 0 ? 0 : nu, kn = K * ns;
        if (ns == 0) {
            if (dets_out) for (int k = 0; k < K; ++k) { dets_out[(s * K + k) * 2] = 1.0; dets_out[(s * K + k) * 2 + 1] = 0.0; }
            continue;
        }
        for (int k = 0; k < K; ++k) {
            for (int io = 0; io < ns; ++io) {
                const int col = k * ns + io;
                for (int jj = 0; jj < ns; ++jj) {
                    const int j = j0 + jj;
                    hd a = P(th, dir, Ly->g[s] + col);
                    for (int u = 0; u < w1; ++u) a = hadd(a, hmul(H1(j, u), P(th, dir, Ly->w[s] + (int64_t)u * kn + col)));
                    hd env = hconst(0.0);
                    for (int m = 0; m < M; ++m) {
                        hd dv[3];
                        for (int q = 0; q < 3; ++q) dv[q] = hsub(x[3 * j + q], hconst(c->nuc_xyz[3 * m + q]));
                        hd sd[3];   /* Sigma (r_j - R_m) */
                        if (c->envelope) {
                            const hd sg = P(th, dir, Ly->sig[s] + (int64_t)col * M + m);
                            for (int p = 0; p < 3; ++p) sd[p] = hmul(sg, dv[p]);
                        } else {
                            for (int p = 0; p < 3; ++p) {
                                int64_t base = Ly->sig[s] + (((int64_t)col * M + m) * 9) + 3 * p;
                                sd[p] = hadd(hadd(hmul(P(th, dir, base + 0), dv[0]), hmul(P(th, dir, base + 1), dv[1])),
                                             hmul(P(th, dir, base + 2), dv[2]));
                            }
                        }
                        hd q = hnorm3(sd[0], sd[1], sd[2]);
                        env = hadd(env, hmul(P(th, dir, Ly->pi[s] + (int64_t)col * M + m), hexp(hscale(q, -1.0))));
                    }
                    S->A[io * ns + jj] = hmul(a, env);
                }
            }
            if (S->mats) {
                const int nmax = nu > nd ? nu : nd;
                double *dst = S->mats + ((size_t)(s * K + k) * nmax * nmax);
                for (int r = 0; r < ns; ++r)
                    for (int q = 0; q < ns; ++q) dst[r * nmax + q] = S->A[r * ns + q].a;
                if (S->mats_b) {
                    double *db = S->mats_b + ((size_t)(s * K + k) * nmax * nmax);
                    for (int r = 0; r < ns; ++r)
                        for (int q = 0; q < ns; ++q) db[r * nmax + q] = S->A[r * ns + q].b;
                }
            }
            int sg; hd la;
            lu_slogdet(ns, S->A, &sg, &la);
            if (dets_out) { dets_out[(s * K + k) * 2] = sg; dets_out[(s * K + k) * 2 + 1] = la.a; }
            sk[k] *= sg;
            lk[k] = hadd(lk[k], la);
        }
    }
    double lmax = -INFINITY;
    for (int k = 0; k < K; ++k)
        if (sk[k] != 0 && lk[k].a > lmax) lmax = lk[k].a;
    if (lmax == -INFINITY) {
        *sign = 0;
        logpsi->a = -INFINITY; logpsi->b = logpsi->c = logpsi->d = NAN;
        return;
    }
    hd sum = hconst(0.0);
    for (int k = 0; k < K; ++k)
        if (sk[k] != 0) sum = hadd(sum, hscale(hexp(hsub(lk[k], hconst(lmax))), (double)sk[k]));
    if (sum.a == 0.0) {
        *sign = 0;
        logpsi->a = -INFINITY; logpsi->b = logpsi->c = logpsi->d = NAN;
        return;
    }
    *sign = sum.a > 0 ? 1 : -1;
    *logpsi = hadd(hconst(lmax), hlogabs(sum));
#undef H1
#undef H1N
#undef H2
#undef H2N
}

/* ------------------------------------------------------------------ */
/* Coulomb terms, brute force                                          */
/* ------------------------------------------------------------------ */
static void coulomb(const orc_cfg *c, const double *x, double *ee, double *en, double *nn)
{
    const int N = c->n_up + c->n_dn, M = c->n_nuc;
    double vee = 0, ven = 0, vnn = 0;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j) {
            double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1], dz = x[3 * i + 2] - x[3 * j + 2];
            vee += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        }
    for (int i = 0; i < N; ++i)
        for (int m = 0; m < M; ++m) {
            double dx = x[3 * i] - c->nuc_xyz[3 * m], dy = x[3 * i + 1] - c->nuc_xyz[3 * m + 1],
                   dz = x[3 * i + 2] - c->nuc_xyz[3 * m + 2];
            ven -= c->nuc_z[m] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    for (int m = 0; m < M; ++m)
        for (int n = m + 1; n < M; ++n) {
            double dx = c->nuc_xyz[3 * m] - c->nuc_xyz[3 * n], dy = c->nuc_xyz[3 * m + 1] - c->nuc_xyz[3 * n + 1],
                   dz = c->nuc_xyz[3 * m + 2] - c->nuc_xyz[3 * n + 2];
            vnn += c->nuc_z[m] * c->nuc_z[n] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    *ee = vee; *en = ven; *nn = vnn;
}

void orc_coulomb(const orc_cfg *c, const double *x, int64_t B, double *parts /*[B][3] ee,en,nn*/)
{
    const int N = c->n_up + c->n_dn;
    for (int64_t w = 0; w < B; ++w) coulomb(c, x + w * 3 * N, &parts[3 * w], &parts[3 * w + 1], &parts[3 * w + 2]);
}

/* ------------------------------------------------------------------ */
/* public entries                                                      */
/* ------------------------------------------------------------------ */
static void load_real(hd *xh, const double *x, int n)
{
    for (int q = 0; q < n; ++q) xh[q] = hconst(x[q]);
}

/* log|psi| and sign for B walkers; theta_dir (may be NULL) gives the
   directional derivative d log|psi| / d theta . dir in dlog (may be NULL). */
void orc_log_psi(const orc_cfg *c, const double *theta, const double *theta_dir, const double *x, int64_t B,
                 double *log_abs, double *sign, double *dlog, double *dets /*[B][2][K][2] or NULL*/,
                 double *h_last /*[B][N][w1] or NULL*/)
{
    orc_layout Ly;
    make_layout(c, &Ly);
    const int N = c->n_up + c->n_dn;
#pragma omp parallel
    {
        scratch S = scratch_alloc(c);
        hd *xh = (hd *)malloc(sizeof(hd) * 3 * N);
        hd *hl = h_last ? (hd *)malloc(sizeof(hd) * (size_t)N * c->w1) : NULL;
        S.hL_out = hl;
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w) {
            load_real(xh, x + w * 3 * N, 3 * N);
            hd lp; int sg;
            eval_walker(c, &Ly, theta, theta_dir, xh, &S, &lp, &sg, dets ? dets + w * 4 * c->n_det : NULL);
            log_abs[w] = lp.a;
            if (sign) sign[w] = sg;
            if (dlog) dlog[w] = lp.b;
            if (hl) for (int q = 0; q < N * c->w1; ++q) h_last[w * N * c->w1 + q] = hl[q].a;
        }
        free(hl);
        free(xh);
        scratch_free(&S);
    }
}

/* local energy (Eq. 2 with the kinetic term of Eq. 3) for B walkers.
   parts [B][4] = kinetic, el-el, nuc-el, nuc-nuc; grad [B][3N] and lap [B]
   (d2 log|psi| summed over coordinates) are optional. */
void orc_local_energy(const orc_cfg *c, const double *theta, const double *x, int64_t B, double *e_loc,
                      double *log_abs, double *parts, double *grad, double *lap)
{
    orc_layout Ly;
    make_layout(c, &Ly);
    const int N = c->n_up + c->n_dn;
#pragma omp parallel
    {
        scratch S = scratch_alloc(c);
        hd *xh = (hd *)malloc(sizeof(hd) * 3 * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w) {
            const double *xw = x + w * 3 * N;
            double sum_g2 = 0.0, sum_d2 = 0.0, lp0 = 0.0;
            int sg = 0;
            for (int cc = 0; cc < 3 * N; ++cc) {
                load_real(xh, xw, 3 * N);
                xh[cc].b = 1.0;
                xh[cc].c = 1.0;
                hd lp;
                eval_walker(c, &Ly, theta, NULL, xh, &S, &lp, &sg, NULL);
                lp0 = lp.a;
                sum_g2 += lp.b * lp.b;
                sum_d2 += lp.d;
                if (grad) grad[w * 3 * N + cc] = lp.b;
            }
            double kin = -0.5 * (sum_d2 + sum_g2);
            double ee, en, nn;
            coulomb(c, xw, &ee, &en, &nn);
            if (sg == 0) kin = NAN;
            e_loc[w] = kin + ee + en + nn;
            if (log_abs) log_abs[w] = sg == 0 ? -INFINITY : lp0;
            if (parts) { parts[4 * w] = kin; parts[4 * w + 1] = ee; parts[4 * w + 2] = en; parts[4 * w + 3] = nn; }
            if (lap) lap[w] = sum_d2;
        }
        free(xh);
        scratch_free(&S);
    }
}

/* orbital matrices A[i][j] = phi_i(r_j) of every (spin, determinant):
   out [B][2][K][nmax][nmax], nmax = max(n_up, n_dn), unused entries 0 */
void orc_orbital_matrices(const orc_cfg *c, const double *theta, const double *x, int64_t B, double *out)
{
    orc_layout Ly;
    make_layout(c, &Ly);
    const int N = c->n_up + c->n_dn;
    const int nmax = c->n_up > c->n_dn ? c->n_up : c->n_dn;
    const size_t per = (size_t)2 * c->n_det * nmax * nmax;
    memset(out, 0, sizeof(double) * per * (size_t)B);
#pragma omp parallel
    {
        scratch S = scratch_alloc(c);
        hd *xh = (hd *)malloc(sizeof(hd) * 3 * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w) {
            load_real(xh, x + w * 3 * N, 3 * N);
            S.mats = out + per * (size_t)w;
            hd lp; int sg;
            eval_walker(c, &Ly, theta, NULL, xh, &S, &lp, &sg, NULL);
        }
        free(xh);
        scratch_free(&S);
    }
}

/* the orbital matrices and their derivative along the parameter direction
   dir (exact, dual numbers): out, out_dir [B][2][K][nmax][nmax] */
void orc_orbital_matrices_dir(const orc_cfg *c, const double *theta, const double *dir, const double *x, int64_t B,
                              double *out, double *out_dir)
{
    orc_layout Ly;
    make_layout(c, &Ly);
    const int N = c->n_up + c->n_dn;
    const int nmax = c->n_up > c->n_dn ? c->n_up : c->n_dn;
    const size_t per = (size_t)2 * c->n_det * nmax * nmax;
    memset(out, 0, sizeof(double) * per * (size_t)B);
    memset(out_dir, 0, sizeof(double) * per * (size_t)B);
#pragma omp parallel
    {
        scratch S = scratch_alloc(c);
        hd *xh = (hd *)malloc(sizeof(hd) * 3 * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w) {
            load_real(xh, x + w * 3 * N, 3 * N);
            S.mats = out + per * (size_t)w;
            S.mats_b = out_dir + per * (size_t)w;
            hd lp; int sg;
            eval_walker(c, &Ly, theta, dir, xh, &S, &lp, &sg, NULL);
        }
        free(xh);
        scratch_free(&S);
    }
}

/* d log|psi| / d theta_i for a list of parameter indices: out [B][n_idx] */
void orc_dlogpsi_dtheta_index(const orc_cfg *c, const double *theta, const int64_t *idx, int64_t n_idx,
                              const double *x, int64_t B, double *out)
{
    orc_layout Ly;
    make_layout(c, &Ly);
    const int N = c->n_up + c->n_dn;
#pragma omp parallel
    {
        scratch S = scratch_alloc(c);
        hd *xh = (hd *)malloc(sizeof(hd) * 3 * N);
        double *dir = (double *)calloc((size_t)Ly.total, sizeof(double));
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int64_t w = 0; w < B; ++w)
            for (int64_t t = 0; t < n_idx; ++t) {
                dir[idx[t]] = 1.0;
                load_real(xh, x + w * 3 * N, 3 * N);
                hd lp; int sg;
                eval_walker(c, &Ly, theta, dir, xh, &S, &lp, &sg, NULL);
                out[w * n_idx + t] = lp.b;
                dir[idx[t]] = 0.0;
            }
        free(dir);
        free(xh);
        scratch_free(&S);
    }
}

/* ------------------------------------------------------------------ */
/* random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)    */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t ctr[4], const uint32_t key[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * ctr[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    ctr[0] = n0; ctr[1] = lo1; ctr[2] = n2; ctr[3] = lo0;
}

void orc_philox4x32_10(const uint32_t counter[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t ctr[4] = {counter[0], counter[1], counter[2], counter[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(ctr, key);
        key[0] += 0x9E3779B9u;
        key[1] += 0xBB67AE85u;
    }
    out[0] = ctr[0]; out[1] = ctr[1]; out[2] = ctr[2]; out[3] = ctr[3];
}

/* uniform in (0, 1] from two words: 53 random bits m, u = (m + 1) 2^-53 */
static double u01(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(m + 1) * 0x1.0p-53;
}

/* normal deviate q of walker w at step `step`, and the accept uniform */
static void draws(uint64_t seed, uint32_t stream_id, int64_t w, uint64_t step, int n3, double *z, double *u)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int q = 0; q < n3; q += 2) {
        uint32_t ctr[4] = {(uint32_t)(q / 2), (uint32_t)w, (uint32_t)step, stream_id}, o[4];
        orc_philox4x32_10(ctr, key, o);
        double u1 = u01(o[0], o[1]), u2 = u01(o[2], o[3]);
        double rad = sqrt(-2.0 * log(u1));
        double ang = 2.0 * M_PI * u2;
        z[q] = rad * cos(ang);
        if (q + 1 < n3) z[q + 1] = rad * sin(ang);
    }
    uint32_t ctr[4] = {0xFFFFFFFFu, (uint32_t)w, (uint32_t)step, stream_id}, o[4];
    orc_philox4x32_10(ctr, key, o);
    *u = u01(o[0], o[1]);
}

void orc_draws(uint64_t seed, uint32_t stream_id, int64_t B, int32_t n3, uint64_t step, double *z /*[B][n3]*/,
               double *u /*[B]*/)
{
    for (int64_t w = 0; w < B; ++w) draws(seed, stream_id, w, step, n3, z + w * n3, u + w);
}

/* the draws of one walker index (any 64-bit value; the counter takes its low
   32 bits), for checking the word-to-deviate map against known answers */
void orc_draw_one(uint64_t seed, uint32_t stream_id, int64_t walker, int32_t n3, uint64_t step, double *z /*[n3]*/,
                  double *u)
{
    draws(seed, stream_id, walker, step, n3, z, u);
}

/*
 * n_steps Metropolis-Hastings moves (Electron Sampler section): all
 * electrons of a walker move together, x' = x + sigma z; the move is kept
 * iff log|psi'| is finite and log u <= 2 (log|psi'| - log|psi|).
 * z_in [n_steps][B][3N] and u_in [n_steps][B] replace the generator when
 * both are given.  x and log_abs are updated in place; n_accept [B] counts.
 */
void orc_metropolis(const orc_cfg *c, const double *theta, double *x, double *log_abs, int64_t B, int32_t n_steps,
                    double sigma, uint64_t seed, uint64_t step0, uint32_t stream_id, const double *z_in,
                    const double *u_in, int32_t *n_accept)
{
    orc_layout Ly;
    make_layout(c, &Ly);
    const int N = c->n_up + c->n_dn, n3 = 3 * N;
#pragma omp parallel
    {
        scratch S = scratch_alloc(c);
        hd *xh = (hd *)malloc(sizeof(hd) * n3);
        double *z = (double *)malloc(sizeof(double) * n3);
        double *xp = (double *)malloc(sizeof(double) * n3);
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w) {
            double *xw = x + w * n3;
            for (int s = 0; s < n_steps; ++s) {
                double u;
                if (z_in && u_in) {
                    memcpy(z, z_in + ((int64_t)s * B + w) * n3, sizeof(double) * n3);
                    u = u_in[(int64_t)s * B + w];
                } else {
                    draws(seed, stream_id, w, step0 + (uint64_t)s, n3, z, &u);
                }
                for (int q = 0; q < n3; ++q) {
                    volatile double step = sigma * z[q]; /* no contraction into an fma */
                    xp[q] = xw[q] + step;
                }
                load_real(xh, xp, n3);
                hd lp; int sg;
                eval_walker(c, &Ly, theta, NULL, xh, &S, &lp, &sg, NULL);
                double lnew = sg == 0 ? -INFINITY : lp.a;
                double A = 2.0 * (lnew - log_abs[w]);
                if (isfinite(lnew) && log(u) <= A) {
                    memcpy(xw, xp, sizeof(double) * n3);
                    log_abs[w] = lnew;
                    if (n_accept) n_accept[w] += 1;
                }
            }
        }
        free(xp); free(z); free(xh);
        scratch_free(&S);
    }
}

int32_t orc_num_threads(void) { return omp_get_max_threads(); }
