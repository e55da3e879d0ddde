/*
 * Test driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only).  TEST INFRASTRUCTURE ONLY:
 * built and run by tests/test_oracle_sanitize.py, never by the library.
 *
 * It compiles the oracle into the same translation unit, reads one case from
 * a binary file and runs every exported oracle call on it, writing the
 * results to a second binary file so the test can compare them with the
 * ordinary build.  Input layout (little endian):
 *   int32 n_nuc, n_up, n_dn, n_layers, w1, w2, n_det, envelope, B, n_idx
 *   double nuc_xyz[3 n_nuc], nuc_z[n_nuc], theta[P], dir[P], x[B][N][3]
 *   int64 idx[n_idx]
 * Output: log_abs, sign, dlog [B] each; e_loc [B]; parts [B][4];
 *   grad [B][3N]; lap [B]; dtheta [B][n_idx]; mats, mats_dir
 *   [B][2][K][nmax][nmax]; coulomb [B][3]; slogdet sign, log [2 B K];
 *   Metropolis x [B][N][3], log_abs [B], n_accept [B] (as doubles).
 */
#include "fn_oracle.c"

#include <stdio.h>

static void *read_n(FILE *f, size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static void put(FILE *f, const double *v, size_t n) { fwrite(v, sizeof(double), n, f); }

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *fi = fopen(argv[1], "rb");
    if (!fi) return 2;
    int32_t *h = (int32_t *)read_n(fi, 10 * sizeof(int32_t));
    orc_cfg c;
    c.n_nuc = h[0]; c.n_up = h[1]; c.n_dn = h[2]; c.n_layers = h[3];
    c.w1 = h[4]; c.w2 = h[5]; c.n_det = h[6]; c.envelope = h[7];
    const int64_t B = h[8], n_idx = h[9];
    const int N = c.n_up + c.n_dn, K = c.n_det, M = c.n_nuc;
    const int nmax = c.n_up > c.n_dn ? c.n_up : c.n_dn;
    double *xyz = (double *)read_n(fi, sizeof(double) * 3 * M);
    double *z = (double *)read_n(fi, sizeof(double) * M);
    c.nuc_xyz = xyz;
    c.nuc_z = z;
    const int64_t P = orc_param_count(&c);
    double *theta = (double *)read_n(fi, sizeof(double) * P);
    double *dir = (double *)read_n(fi, sizeof(double) * P);
    double *x = (double *)read_n(fi, sizeof(double) * B * N * 3);
    int64_t *idx = (int64_t *)read_n(fi, sizeof(int64_t) * n_idx);
    fclose(fi);

    double *la = malloc(sizeof(double) * B), *sg = malloc(sizeof(double) * B), *dl = malloc(sizeof(double) * B);
    double *dets = malloc(sizeof(double) * B * 2 * K * 2);
    double *hl = malloc(sizeof(double) * B * N * c.w1);
    orc_log_psi(&c, theta, dir, x, B, la, sg, dl, dets, hl);
    double *e = malloc(sizeof(double) * B), *la2 = malloc(sizeof(double) * B), *parts = malloc(sizeof(double) * B * 4);
    double *gr = malloc(sizeof(double) * B * 3 * N), *lap = malloc(sizeof(double) * B);
    orc_local_energy(&c, theta, x, B, e, la2, parts, gr, lap);
    double *dt = malloc(sizeof(double) * B * (n_idx ? n_idx : 1));
    orc_dlogpsi_dtheta_index(&c, theta, idx, n_idx, x, B, dt);
    const size_t nm = (size_t)B * 2 * K * nmax * nmax;
    double *mats = malloc(sizeof(double) * nm), *mats2 = malloc(sizeof(double) * nm), *matd = malloc(sizeof(double) * nm);
    orc_orbital_matrices(&c, theta, x, B, mats);
    orc_orbital_matrices_dir(&c, theta, dir, x, B, mats2, matd);
    double *cou = malloc(sizeof(double) * B * 3);
    orc_coulomb(&c, x, B, cou);
    /* the up-spin matrices of every determinant through the exported slogdet */
    double *ss = malloc(sizeof(double) * 2 * B * K), *sl = malloc(sizeof(double) * 2 * B * K);
    double *up = malloc(sizeof(double) * B * K * (c.n_up ? c.n_up * c.n_up : 1));
    for (int64_t w = 0; w < B; ++w)
        for (int k = 0; k < K; ++k)
            for (int r = 0; r < c.n_up; ++r)
                for (int q = 0; q < c.n_up; ++q)
                    up[((w * K + k) * c.n_up + r) * c.n_up + q] = mats[(((w * 2 + 0) * K + k) * nmax + r) * nmax + q];
    if (c.n_up) orc_slogdet(c.n_up, B * K, up, ss, sl);
    else for (int64_t t = 0; t < B * K; ++t) { ss[t] = 1.0; sl[t] = 0.0; }
    double *xm = malloc(sizeof(double) * B * N * 3), *lm = malloc(sizeof(double) * B);
    int32_t *acc = calloc((size_t)B, sizeof(int32_t));
    memcpy(xm, x, sizeof(double) * B * N * 3);
    memcpy(lm, la, sizeof(double) * B);
    orc_metropolis(&c, theta, xm, lm, B, 3, 0.2, 7, 0, 2, NULL, NULL, acc);
    double *accd = malloc(sizeof(double) * B);
    for (int64_t w = 0; w < B; ++w) accd[w] = acc[w];

    FILE *fo = fopen(argv[2], "wb");
    if (!fo) return 2;
    put(fo, la, B); put(fo, sg, B); put(fo, dl, B);
    put(fo, e, B); put(fo, parts, B * 4); put(fo, gr, B * 3 * N); put(fo, lap, B);
    put(fo, dt, B * n_idx);
    put(fo, mats, nm); put(fo, matd, nm);
    put(fo, cou, B * 3);
    put(fo, ss, B * K); put(fo, sl, B * K);
    put(fo, xm, B * N * 3); put(fo, lm, B); put(fo, accd, B);
    fclose(fo);
    free(h); free(xyz); free(z); free(theta); free(dir); free(x); free(idx);
    free(la); free(sg); free(dl); free(dets); free(hl); free(e); free(la2); free(parts); free(gr); free(lap);
    free(dt); free(mats); free(mats2); free(matd); free(cou); free(ss); free(sl); free(up); free(xm); free(lm);
    free(acc); free(accd);
    return 0;
}
