/* Drives every entry point of the CPU oracle once, for a build with the
 * address and undefined-behaviour sanitizers (tests only).  The oracle is
 * included as one translation unit so its types are visible here. */
#include "../../oracle/srm_oracle.c"

#include <stdio.h>

/* xorshift64* points in [0, L): test inputs only, not part of the method */
static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    rs ^= rs >> 12; rs ^= rs << 25; rs ^= rs >> 27;
    return (double)((rs * 0x2545F4914F6CDD1Dull) >> 11) * 0x1p-53;
}

static int run_case(int dim, int shape, int64_t n, int poly, double box_z)
{
    o_state st;
    memset(&st, 0, sizeof st);
    o_params *p = &st.p;
    p->dim = dim; p->shape = shape; p->n = n;
    p->box[0] = 1.0; p->box[1] = 0.9; p->box[2] = box_z;
    double vol = (dim == 3) ? 0.9 * box_z : 0.9;
    int disk = shape == O_PLATELET || shape == O_SPHERODISK;
    double tr = shape == O_SPHERODISK ? 0.1 : 0.01;
    double f = disk ? 0.01 : 0.3;
    double coeff = disk ? 2.0 * M_PI * tr : (dim == 2 ? M_PI : 4.0 * M_PI / 3.0);
    p->s_target = pow(f * vol / (coeff * (double)n), 1.0 / dim);
    p->c_w = 0.05; p->c_m = 0.1 * p->s_target; p->c_n = 0.1; p->thick_ratio = tr;
    p->n_k = 4; p->n_l = 6; p->seed = 77;
    st.pos = (double *)calloc(3 * (size_t)n, sizeof(double));
    st.nrm = disk ? (double *)calloc(3 * (size_t)n, sizeof(double)) : NULL;
    double *rho = poly ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < dim; ++a) st.pos[3 * i + a] = urand() * p->box[a];
        if (st.nrm) {
            double v[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5};
            double q = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            for (int a = 0; a < 3; ++a) st.nrm[3 * i + a] = v[a] / q;
        }
        if (rho) rho[i] = 0.8 + 0.4 * urand();
    }
    st.rho = rho;
    int64_t sweeps = 0, passes = 0;
    int rc = o_run(&st, 400, &sweeps, &passes);
    if (rc != O_OK && rc != O_ENOTCONV) return 1;
    int64_t na[3]; double inv_w[3];
    o_grid(p, st.s * o_rho_max(&st), na, inv_w);
    int32_t ov = 0;
    uint8_t *acc = (uint8_t *)malloc((size_t)n);
    uint8_t *mask = (uint8_t *)calloc((size_t)(na[0] * na[1] * na[2]), 1);
    mask[0] = 1;
    if (o_pass(&st, na, inv_w, st.s, O_SHAKE, 1, acc, mask, &ov)) return 1;
    if (o_overlap(&st, na, inv_w, st.s, &ov)) return 1;
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    o_bin(p, na, inv_w, st.pos, cell);
    int64_t cnt = o_pairs_brute(&st, st.s, 0.01, 0, NULL);
    int32_t *ij = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(cnt + 1));
    o_pairs_brute(&st, st.s, 0.01, cnt, ij);
    int32_t mask_p = 0;
    if (o_percolation(&st, st.s, 0.02, &mask_p)) return 1;
    if (shape == O_BALL) {
        uint64_t counts[16];
        double *dist = (double *)malloc(sizeof(double) * (size_t)n);
        if (o_rdf_brute(&st, 16, 0.2, counts) || o_nearest_brute(&st, 0.2, dist)) return 1;
        o_softrdf_params sp = {dim, 16, {p->box[0], p->box[1], p->box[2]}, 5.0 * p->s_target, 1.0};
        double *pos_soa = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        double *radii = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) pos_soa[3 * i + a] = st.pos[3 * i + a];
            radii[i] = rho ? st.s * rho[i] : st.s;
        }
        double g[16], e = 0.0, dg[16];
        for (int b = 0; b < 16; ++b) dg[b] = 0.1 * b;
        o_softrdf_fwd(&sp, n, pos_soa, radii, g, &e);
        double *gp = (double *)calloc(3 * (size_t)n, sizeof(double));
        double *gr = (double *)calloc((size_t)n, sizeof(double));
        o_softrdf_grad(&sp, n, pos_soa, radii, dg, 1.0, gp, gr);
        free(dist); free(pos_soa); free(radii); free(gp); free(gr);
    }
    printf("dim %d shape %d n %lld poly %d: rc %d sweeps %lld passes %lld pairs %lld\n", dim,
           shape, (long long)n, poly, rc, (long long)sweeps, (long long)passes, (long long)cnt);
    free(st.pos); free(st.nrm); free(rho); free(acc); free(mask); free(cell); free(ij);
    return 0;
}

int main(void)
{
    int bad = 0;
    bad |= run_case(2, O_BALL, 500, 0, 1.0);
    bad |= run_case(2, O_BALL, 400, 1, 1.0);
    bad |= run_case(3, O_BALL, 600, 0, 1.2);
    bad |= run_case(3, O_BALL, 500, 1, 0.8);
    bad |= run_case(3, O_PLATELET, 300, 0, 1.0);
    bad |= run_case(3, O_SPHERODISK, 300, 0, 1.0);
    bad |= run_case(3, O_SPHERODISK, 200, 1, 0.9);
    bad |= run_case(2, O_BALL, 1, 0, 1.0);
    /* RSA, balls and platelets, and a budget that runs out */
    double box[3] = {1.0, 1.0, 1.0};
    for (int shape = 0; shape < 2; ++shape) {
        int64_t n = 800, drawn = 0, placed = 0;
        double *pos = (double *)calloc(3 * (size_t)n, sizeof(double));
        double *nrm = shape ? (double *)calloc(3 * (size_t)n, sizeof(double)) : NULL;
        int64_t *src = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        int rc = o_rsa(3, shape, n, box, 0.03, 5, 100000, pos, nrm, src, &drawn, &placed);
        int rc2 = o_rsa(3, shape, n, box, 0.03, 5, 50, pos, nrm, src, &drawn, &placed);
        if (rc != O_OK || rc2 != O_ENOTCONV) bad = 1;
        free(pos); free(nrm); free(src);
    }
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
