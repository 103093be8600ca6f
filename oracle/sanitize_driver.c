/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE: drives every entry point of the
 * FP64 oracle on small synthetic problems so that the oracle can be built and
 * run under AddressSanitizer and UndefinedBehaviorSanitizer (host code only;
 * tests/test_oracle_sanitizers.py compiles and runs it).  The inputs are a
 * jittered lattice from a fixed linear congruential sequence: this program
 * checks memory safety and defined behaviour, not physics (the pins do that).
 * Exit status 0 when every call returned and each photon ledger closed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "traphic_oracle.h"

static uint64_t lcg = 88172645463325252ull;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int run(int recomb_mode, int n_side, int two_instances)
{
    const double kpc = 3.0857e21, L = 6.6 * kpc;
    const int n1 = n_side * n_side * n_side, n_inst = two_instances ? 2 : 1;
    const int N = n1 * n_inst;
    double *pos = malloc(sizeof(double) * 3 * N), *nH = malloc(sizeof(double) * N), *NH = malloc(sizeof(double) * N);
    double *xHI = malloc(sizeof(double) * N), *T = malloc(sizeof(double) * N);
    double box[12];
    int64_t off[3] = {0, n1, 2 * (int64_t)n1};
    for (int k = 0; k < n_inst; ++k) {
        for (int a = 0; a < 3; ++a) {
            box[6 * k + a] = 3.0 * L * k * (a == 0);
            box[6 * k + 3 + a] = box[6 * k + a] + L;
        }
        const double dx = L / n_side;
        for (int i = 0; i < n1; ++i) {
            const int g[3] = {i / (n_side * n_side), (i / n_side) % n_side, i % n_side};
            const int64_t j = (int64_t)k * n1 + i;
            for (int a = 0; a < 3; ++a) pos[3 * j + a] = box[6 * k + a] + (g[a] + 0.5 + 0.6 * (unif() - 0.5)) * dx;
            nH[j] = 1e-3 * (0.5 + unif());
            NH[j] = nH[j] * dx * dx * dx;
            xHI[j] = 0.2 + 0.8 * unif();
            T[j] = 1e4;
        }
    }
    or_params p = {0};
    p.n_ngb = 16;
    p.n_tc = 8;
    p.n_rc = 8;
    p.n_ec = 8;
    p.n_freq = 2;
    p.rr_bin = 1;
    p.recomb_mode = recomb_mode;
    p.isothermal = 0;
    p.n_em = 2;
    p.max_hops = 400;
    p.max_vip_depth = 4;
    p.dt = 0.5 * 3.1536e13;
    p.floor_rel = 1e-20;
    p.chem_frac = 0.1;
    p.seed = 1311018299ull;
    const double sigma[2] = {6.3e-18, 6.3e-18}, eps[2] = {3.0 * 1.602e-12, 2.3 * 1.602e-12};
    or_sim *S = or_create(&p, sigma, eps, n_inst, off, box, pos, nH, NH, xHI, T);
    if (!S) {
        fprintf(stderr, "or_create: %s\n", or_error());
        return 1;
    }
    int32_t inst[2] = {0, 1}, kind[2] = {OR_SRC_POINT, OR_SRC_PLANE_XLO}, nside[2] = {0, 5};
    double spos[6] = {L / 2, L / 2, L / 2, 0, 0, 0}, rate[4] = {5e48, 0.0, 1e6, 0.0};
    if (or_add_sources(S, n_inst, inst, kind, spos, rate, nside)) {
        fprintf(stderr, "or_add_sources: %s\n", or_error());
        return 1;
    }
    if (two_instances) {
        /* a barrier disk in the first instance, across the point source's light */
        const double bc[3] = {0.4 * L, L / 2, L / 2};
        if (or_set_barrier(S, 0, bc, 0.2 * L)) {
            fprintf(stderr, "or_set_barrier: %s\n", or_error());
            return 1;
        }
    }
    or_step(S, 3);
    const int nf = 2, G = 16;
    double *x = malloc(sizeof(double) * N), *t = malloc(sizeof(double) * N), *A = malloc(sizeof(double) * N * nf);
    double *P = malloc(sizeof(double) * N * nf), led[2 * 2 * 5];
    int64_t cnt[4];
    or_get_state(S, x, t, A, P, led, cnt);
    double *bN = malloc(sizeof(double) * N * G), *bd = malloc(sizeof(double) * 3 * N * G), *bc = malloc(sizeof(double) * N * G);
    or_get_bins(S, bN, bd, bc);
    uint64_t *mask = malloc(sizeof(uint64_t) * N * G);
    or_cone_masks(S, mask);
    int32_t *ngb = malloc(sizeof(int32_t) * N * 16);
    double *h = malloc(sizeof(double) * N);
    or_get_ngb(S, ngb, h);
    const int64_t ne = or_n_emitters(S);
    int32_t *engb = malloc(sizeof(int32_t) * (ne + 1) * 16);
    double *eh = malloc(sizeof(double) * (ne + 1));
    or_get_emitter_ngb(S, engb, eh);
    double *nrr = malloc(sizeof(double) * N);
    or_get_nrr(S, nrr);
    double q[6] = {L / 3, L / 2, L / 2, L / 2, L / 3, L / 4};
    int32_t qn[32];
    double qh[2];
    or_knn_points(S, 0, 2, q, qn, qh);
    double d[3] = {1.0, 0.3, -0.2}, xv[3] = {L / 3 + 0.2 * kpc, L / 2, L / 2}, dep[16], nhi, l, nabs, nrem, hv;
    or_vip_leg(S, 0, q, xv, d, 1e55, 0, qn, &hv, dep, &nhi, &l, &nabs, &nrem);
    double prof[20 * 2];
    int64_t pc[20];
    const double c0[3] = {L / 2, L / 2, L / 2}, ax[3] = {1, 0, 0};
    or_shell_profile(n1, nf, pos, P, p.dt, c0, NULL, 0.0, L / 2, 20, 0, 1.0, prof, pc);
    or_shell_profile(n1, nf, pos, P, p.dt, c0, ax, L / 4, L / 2, 20, 1, 3.0, prof, pc);
    int bad = 0;
    for (int k = 0; k < n_inst; ++k)
        for (int nu = 0; nu < nf; ++nu) {
            const double *e = led + (k * nf + nu) * 5;
            if (e[0] > 0 && fabs(e[0] - e[1] - e[2] - e[3] - e[4]) > 1e-12 * e[0]) bad = 1;
        }
    or_destroy(S);
    free(pos), free(nH), free(NH), free(xHI), free(T), free(x), free(t), free(A), free(P);
    free(bN), free(bd), free(bc), free(mask), free(ngb), free(h), free(engb), free(eh), free(nrr);
    return bad;
}

int main(void)
{
    /* primitives */
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    or_philox4x32_10(ctr, key, out);
    double u[3 * 16], R[9], v[3] = {1, 1, 0}, dd[3] = {1, 0, 0}, pp[3];
    or_dirset(16, u);
    or_rotation(7, 1, 2, 3, 4, R);
    (void)or_in_cone(v, dd, 8);
    double rt[8];
    or_rates(2e4, rt);
    or_params cp = {0};
    cp.n_freq = 1;
    cp.recomb_mode = OR_RR_TRANSPORT;
    cp.dt = 3.1536e12;
    cp.chem_frac = 0.1;
    double eps = 1e-12, Ab = 1e55, xh = 0.5, Tt = 1e4, rr = 0;
    int64_t ns = 0;
    or_chem_one(&cp, &eps, &Ab, 1e-3, 1e60, &xh, &Tt, &rr, &ns);
    (void)or_vip_sample(7, 2, 3, 4, 5, dd, 8, pp);
    double N2[2] = {1, 2}, d2[6] = {1, 0, 0, 0, 1, 0}, c2[2] = {0, 1}, oN, od[3], oc;
    or_merge_packets(2, N2, d2, c2, &oN, od, &oc);
    const double la[3] = {-1, 0, 0}, lb[3] = {1, 0.5, 0}, lc[3] = {0, 0, 0};
    (void)or_leg_crosses_disk(la, lb, lc, 1.0);
    /* one instance with a point source; two instances, the second lit by a plane front */
    int bad = run(OR_RR_TRANSPORT, 6, 0) | run(OR_RR_ORIGINAL, 5, 0) | run(OR_CASE_A_NO_RR, 4, 0) |
              run(OR_CASE_B_OTS, 5, 1) | run(OR_RR_TRANSPORT, 5, 1);
    printf(bad ? "ledger mismatch\n" : "sanitize driver OK\n");
    return bad;
}
