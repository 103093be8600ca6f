/*
 * traphic_oracle.c -- plain FP64 CPU oracle of one TRAPHIC radiative-transfer
 * step with recombination radiation (RR) transported in reception cones.
 *
 * TEST INFRASTRUCTURE ONLY: the slow reference that the HIP library is checked
 * against.  It shares no code with the HIP library.  Only tests/, the smoke
 * check and the benchmark's CPU-baseline leg may load it.
 *
 * Everything is written in the order the paper describes the method
 * (section 2.1 "TRAPHIC", section 2.2 "Implementation of recombination
 * radiation").  Details the paper leaves to its predecessor papers are filled
 * in by documented readings; each such place says "Reading:".
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math, no
 * OpenMP, so that libm calls are the scalar glibc ones).
 */
#include "traphic_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define C_LIGHT 2.99792458e10 /* cm/s */
#define K_BOLTZ 1.380649e-16  /* erg/K */
#define T_HI 157807.0         /* K, hydrogen ionization potential / k_B */
#define T_CMB 2.725           /* K, CMB temperature today (Compton cooling) */
#define MAX_SUBSTEPS 1000000
#define VIP_MAX_ATTEMPTS 65536

/* Philox counter tags: what a random draw is for. */
enum { TAG_RC = 1, TAG_EC = 2, TAG_VIP_T = 3, TAG_VIP_E = 4, TAG_RR_EC = 5, TAG_VIP_RR = 6 };

static char g_err[256];
const char *or_error(void) { return g_err; }
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011, "Parallel random numbers: */
/* as easy as 1, 2, 3"): 10 rounds of a multiply-xor bijection keyed by a      */
/* Weyl sequence.  Used for every random draw the method makes: rotations of  */
/* the emission and reception directions and virtual-particle positions.     */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Four uniforms on (-1, 1) from one Philox block, each exactly representable. */
static void draw4(uint64_t seed, uint32_t tag, uint32_t attempt, uint32_t step, uint32_t a,
                  uint32_t b, double u[4])
{
    uint32_t ctr[4] = {tag | (attempt << 4), step, a, b};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    for (int i = 0; i < 4; ++i) {
        double v = ((double)w[i] + 0.5) * (1.0 / 4294967296.0);
        u[i] = 2.0 * v - 1.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Isotropic direction sets (section 2.1: N_EC emission directions, N_RC     */
/* reception directions).  Reading: 8 directions are the cube diagonals      */
/* (their Voronoi cells are exactly the octants); other even counts use the   */
/* spherical Fibonacci lattice on one hemisphere mirrored through the centre. */
/* ------------------------------------------------------------------------ */
void or_dirset(int32_t n, double *u)
{
    if (n == 8) {
        double s = 1.0 / sqrt(3.0);
        for (int k = 0; k < 8; ++k) {
            u[3 * k + 0] = (k & 4) ? -s : s;
            u[3 * k + 1] = (k & 2) ? -s : s;
            u[3 * k + 2] = (k & 1) ? -s : s;
        }
        return;
    }
    /* Fibonacci points of the upper hemisphere plus their antipodes (for even
     * n), so that the set has no net direction, as isotropic emission needs. */
    double ga = M_PI * (3.0 - sqrt(5.0));
    int half = (n % 2 == 0) ? n / 2 : n;
    for (int k = 0; k < half; ++k) {
        double z = 1.0 - (2.0 * k + 1.0) / (double)n;
        double r = sqrt(1.0 - z * z);
        double ph = ga * (double)k;
        u[3 * k + 0] = r * cos(ph);
        u[3 * k + 1] = r * sin(ph);
        u[3 * k + 2] = z;
    }
    for (int k = half; k < n; ++k) {
        u[3 * k + 0] = -u[3 * (k - half) + 0];
        u[3 * k + 1] = -u[3 * (k - half) + 1];
        u[3 * k + 2] = -u[3 * (k - half) + 2];
    }
}

/* Uniform random rotation (section 2.1: directions are randomly rotated before
 * each emission; reception directions are rotated frequently).  A point drawn
 * uniformly in the 4-ball and normalised is a uniform unit quaternion, hence a
 * Haar-uniform rotation.  Only + - * / sqrt are used. */
void or_rotation(uint64_t seed, uint32_t tag, uint32_t step, uint32_t a, uint32_t b, double R[9])
{
    double q[4];
    double s = 0.0;
    for (uint32_t att = 0;; ++att) {
        draw4(seed, tag, att, step, a, b, q);
        s = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (s <= 1.0 && s >= 1e-6) break;
    }
    double n = sqrt(s);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void rotate(const double R[9], const double u[3], double out[3])
{
    out[0] = R[0] * u[0] + R[1] * u[1] + R[2] * u[2];
    out[1] = R[3] * u[0] + R[4] * u[1] + R[5] * u[2];
    out[2] = R[6] * u[0] + R[7] * u[1] + R[8] * u[2];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Transmission cone (section 2.1): a regular cone of solid angle 4 pi / N_TC
 * around the propagation direction d, i.e. half-angle theta with
 * cos(theta) = 1 - 2/N_TC.  v lies in it iff v.d > 0 and
 * (v.d)^2 >= cos^2(theta) |v|^2 |d|^2.  Reading: the boundary is inclusive. */
int or_in_cone(const double v[3], const double d[3], int32_t n_tc)
{
    double c = 1.0 - 2.0 / (double)n_tc;
    double a = dot3(v, d);
    if (!(a > 0.0)) return 0;
    return a * a >= c * c * dot3(v, v) * dot3(d, d);
}

/* Index of the direction in set w (n entries) closest to d: max dot product,
 * ties to the lower index.  Used for reception-cone binning (section 2.1) and
 * for the Voronoi emission cones (reading). */
static int nearest_dir(const double *w, int n, const double d[3])
{
    int best = 0;
    double bv = dot3(d, w);
    for (int k = 1; k < n; ++k) {
        double v = dot3(d, w + 3 * k);
        if (v > bv) {
            bv = v;
            best = k;
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Rate coefficients (section 2.1: recombination fits of Hui & Gnedin 1997;   */
/* collisional ionization and cooling as in the pawlik2011 tables, which are  */
/* not reproduced in the paper).  Reading: the Hui & Gnedin (1997) fits for   */
/* alpha_A, alpha_B, collisional ionization and recombination cooling; Cen    */
/* (1992) collisional excitation; free-free with Gaunt factor 1.3; Compton    */
/* cooling off the z = 0 CMB.                                                 */
/* out: alpha_A, alpha_B, beta, recA cool, recB cool, coll.exc. cool,         */
/*      free-free cool, Compton coefficient (all cgs).                        */
/* ------------------------------------------------------------------------ */
void or_rates(double T, double out[8])
{
    double lam = 2.0 * T_HI / T;
    out[0] = 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
    out[1] = 2.753e-14 * pow(lam, 1.500) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
    out[2] = 21.11 * pow(T, -1.5) * exp(-lam / 2.0) * pow(lam, -1.089) /
             pow(1.0 + pow(lam / 0.354, 0.874), 1.101);
    out[3] = 1.778e-29 * T * pow(lam, 1.965) / pow(1.0 + pow(lam / 0.541, 0.502), 2.697);
    out[4] = 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam / 2.250, 0.376), 3.720);
    out[5] = 7.5e-19 * exp(-118348.0 / T) / (1.0 + sqrt(T / 1e5));
    out[6] = 1.42e-27 * 1.3 * sqrt(T);
    out[7] = 1.017e-37 * pow(T_CMB, 4.0) * (T - T_CMB);
}

/* ------------------------------------------------------------------------ */
/* Chemistry step of one particle (section 2.1: Gamma_nu = N_abs,nu /        */
/* (N_HI dt), heating Gamma_nu <eps>_nu, then x and T updated over dt;       */
/* section 2.2: case A with RR transport, RR photons from recombinations to   */
/* the ground state, alpha_1 = alpha_A - alpha_B).                            */
/* Reading: the neutral fraction y follows dy/dt = alpha n_e (1-y) -         */
/* (Gamma + beta n_e) y, integrated with backward Euler (rates frozen over a */
/* sub-step); the sub-step is limited so that y changes by at most chem_frac */
/* of min(y, 1-y) (floored at 1e-6) and T by chem_frac of itself.  With      */
/* photoheating and cooling d[(1+x)T]/dt = 2 (H - Lambda)/(3 k n_H), where   */
/* H = n_H y sum_nu Gamma_nu <eps>_nu with the current y.                     */
/* ------------------------------------------------------------------------ */
void or_chem_one(const or_params *p, const double *eps, const double *A, double nH, double NH,
                 double *xHI, double *T, double *nrr, int64_t *nsub)
{
    int nf = p->n_freq;
    double dt = p->dt;
    double y = *xHI;
    double NHI0 = y * NH;
    double Asum = 0.0, Esum = 0.0;
    for (int nu = 0; nu < nf; ++nu) {
        Asum += A[nu];
        Esum += A[nu] * eps[nu];
    }
    double gam = NHI0 > 0.0 ? Asum / (NHI0 * dt) : 0.0;
    /* photoheating per HI atom sum_nu Gamma_nu <eps>_nu (section 2.1); per    */
    /* volume it scales with the neutral density n_H y as y evolves, like the  */
    /* photoionizations                                                         */
    double heat_y = NHI0 > 0.0 ? Esum / (NHI0 * dt) * nH : 0.0;
    int caseB = p->recomb_mode == OR_CASE_B_OTS;
    double Tc = *T;
    double t = 0.0, rr = 0.0;
    int64_t n = 0;
    double rt[8];
    while (t < dt && n < MAX_SUBSTEPS) {
        or_rates(Tc, rt);
        double alpha = caseB ? rt[1] : rt[0];
        double x = 1.0 - y;
        double ne = nH * x;
        double ion = gam + rt[2] * ne;
        double rec = alpha * ne;
        double dydt = rec * x - ion * y;
        double dts = dt - t;
        double s = y < x ? y : x;
        if (s < 1e-6) s = 1e-6;
        if (fabs(dydt) > 0.0) {
            double lim = p->chem_frac * s / fabs(dydt);
            if (lim < dts) dts = lim;
        }
        double dY = 0.0, Y = 0.0;
        if (!p->isothermal) {
            double nHI = nH * y, nHII = nH * x;
            double lam_cool = (caseB ? rt[4] : rt[3]) * ne * nHII + K_BOLTZ * T_HI * rt[2] * ne * nHI +
                              rt[5] * ne * nHI + rt[6] * ne * nHII + rt[7] * ne;
            dY = 2.0 * (heat_y * y - lam_cool) / (3.0 * K_BOLTZ * nH);
            Y = (1.0 + x) * Tc;
            if (fabs(dY) > 0.0) {
                double limT = p->chem_frac * Y / fabs(dY);
                if (limT < dts) dts = limT;
            }
        }
        double yn = (y + dts * rec) / (1.0 + dts * (ion + rec));
        if (p->recomb_mode == OR_RR_TRANSPORT || p->recomb_mode == OR_RR_ORIGINAL)
            rr += (rt[0] - rt[1]) * ne * (1.0 - yn) * NH * dts;
        if (!p->isothermal) {
            Y = Y + dts * dY;
            Tc = Y / (2.0 - yn);
            if (Tc < 10.0) Tc = 10.0;
        }
        y = yn;
        t += dts;
        ++n;
    }
    *xHI = y;
    *T = Tc;
    *nrr = rr;
    if (nsub) *nsub = n;
}

/* ------------------------------------------------------------------------ */
/* Simulation state                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t inst, kind, src;
    double pos[3];
    double *pk; /* photons per packet and bin for one emission sub-step */
    int32_t *ngb;
    double h;
} emitter;

typedef struct {
    int32_t nc[3];
    double lo[3], cs[3];
    int64_t cell0;
} grid;

struct or_sim {
    or_params p;
    int G, nf;
    int64_t N;
    int32_t n_inst;
    int64_t *inst_off;
    double *box;
    int32_t *inst_of;
    double *sigma, *eps;
    double *pos, *nH, *NH, *xHI, *T, *h;
    int32_t *ngb;
    double *u_rc, *u_ec;
    double *bN, *bd, *bc;       /* packet bins [N][n_freq][n_rc] */
    double *aN, *aS, *aC;       /* merge accumulators, same layout */
    unsigned char *keep;        /* 1 while a bin holds only its own staying packet */
    double *A, *P;              /* absorbed / passing photons of the current step */
    double *nrr;                /* RR photons awaiting emission at the next step */
    double *led;                /* [n_inst][n_freq][4] cumulative E, A, X, R */
    int64_t counters[4];        /* steps, hops, virtual particles, packet updates */
    int64_t n_emit;
    emitter *em;
    grid *gr;
    int64_t *cell_start;
    int64_t *cell_idx;
    double rc_rot[9];
    double *w_rc;               /* rotated reception directions of this step */
    double *barrier;            /* [n_inst][4]: centre and radius of a barrier disk (radius 0: none) */
};

static void *xcalloc(size_t n, size_t s)
{
    void *q = calloc(n ? n : 1, s);
    if (!q) {
        fprintf(stderr, "oracle: out of memory\n");
        abort();
    }
    return q;
}

/* --- uniform cell grid per instance, used only to find nearest neighbours --- */
static void build_grid(or_sim *S)
{
    S->gr = xcalloc((size_t)S->n_inst, sizeof(grid));
    int64_t ncell = 0;
    for (int k = 0; k < S->n_inst; ++k) {
        grid *g = &S->gr[k];
        int64_t n = S->inst_off[k + 1] - S->inst_off[k];
        double L[3], vol = 1.0;
        for (int a = 0; a < 3; ++a) {
            L[a] = S->box[6 * k + 3 + a] - S->box[6 * k + a];
            vol *= L[a];
            g->lo[a] = S->box[6 * k + a];
        }
        double cs = cbrt(2.0 * vol / (double)n);
        for (int a = 0; a < 3; ++a) {
            int m = (int)(L[a] / cs);
            if (m < 1) m = 1;
            if (m > 1024) m = 1024;
            g->nc[a] = m;
            g->cs[a] = L[a] / m;
        }
        g->cell0 = ncell;
        ncell += (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
    }
    int64_t *cnt = xcalloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cid = xcalloc((size_t)S->N, sizeof(int64_t));
    for (int64_t i = 0; i < S->N; ++i) {
        grid *g = &S->gr[S->inst_of[i]];
        int c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (int)floor((S->pos[3 * i + a] - g->lo[a]) / g->cs[a]);
            if (c[a] < 0) c[a] = 0;
            if (c[a] >= g->nc[a]) c[a] = g->nc[a] - 1;
        }
        cid[i] = g->cell0 + ((int64_t)c[0] * g->nc[1] + c[1]) * g->nc[2] + c[2];
        cnt[cid[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cnt[c + 1] += cnt[c];
    S->cell_start = cnt;
    S->cell_idx = xcalloc((size_t)S->N, sizeof(int64_t));
    int64_t *fill = xcalloc((size_t)ncell, sizeof(int64_t));
    for (int64_t i = 0; i < S->N; ++i) S->cell_idx[cnt[cid[i]] + fill[cid[i]]++] = i;
    free(fill);
    free(cid);
}

/* Keep the K smallest (distance^2, index) pairs in ascending order. */
static void knn_insert(double *bd, int64_t *bi, int *cnt, int K, double d2, int64_t j)
{
    if (*cnt == K) {
        double ld = bd[K - 1];
        if (d2 > ld || (d2 == ld && j > bi[K - 1])) return;
    }
    int pos = (*cnt < K) ? (*cnt)++ : K - 1;
    while (pos > 0 && (bd[pos - 1] > d2 || (bd[pos - 1] == d2 && bi[pos - 1] > j))) {
        bd[pos] = bd[pos - 1];
        bi[pos] = bi[pos - 1];
        --pos;
    }
    bd[pos] = d2;
    bi[pos] = j;
}

/* The K nearest particles of instance k to point x (excluding index self),
 * ordered by (distance^2, index); distance^2 = (dx dx + dy dy) + dz dz with
 * d = x_j - x.  Section 2.1: packets are handed to the neighbours inside the
 * smoothing volume; reading: the smoothing volume holds exactly the N_ngb
 * nearest particles and h is the distance to the farthest of them. */
static void knn(const or_sim *S, int k, const double x[3], int64_t self, int K, int32_t *out,
                double *h)
{
    const grid *g = &S->gr[k];
    double bd[64];
    int64_t bi[64];
    int cnt = 0;
    int c[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = (int)floor((x[a] - g->lo[a]) / g->cs[a]);
        if (c[a] < 0) c[a] = 0;
        if (c[a] >= g->nc[a]) c[a] = g->nc[a] - 1;
    }
    double csmin = g->cs[0];
    if (g->cs[1] < csmin) csmin = g->cs[1];
    if (g->cs[2] < csmin) csmin = g->cs[2];
    int smax = g->nc[0];
    if (g->nc[1] > smax) smax = g->nc[1];
    if (g->nc[2] > smax) smax = g->nc[2];
    for (int s = 0; s <= smax; ++s) {
        for (int ix = c[0] - s; ix <= c[0] + s; ++ix) {
            if (ix < 0 || ix >= g->nc[0]) continue;
            for (int iy = c[1] - s; iy <= c[1] + s; ++iy) {
                if (iy < 0 || iy >= g->nc[1]) continue;
                for (int iz = c[2] - s; iz <= c[2] + s; ++iz) {
                    if (iz < 0 || iz >= g->nc[2]) continue;
                    int cheb = abs(ix - c[0]);
                    if (abs(iy - c[1]) > cheb) cheb = abs(iy - c[1]);
                    if (abs(iz - c[2]) > cheb) cheb = abs(iz - c[2]);
                    if (cheb != s) continue;
                    int64_t cell = g->cell0 + ((int64_t)ix * g->nc[1] + iy) * g->nc[2] + iz;
                    for (int64_t t = S->cell_start[cell]; t < S->cell_start[cell + 1]; ++t) {
                        int64_t j = S->cell_idx[t];
                        if (j == self) continue;
                        double dx = S->pos[3 * j + 0] - x[0];
                        double dy = S->pos[3 * j + 1] - x[1];
                        double dz = S->pos[3 * j + 2] - x[2];
                        double d2 = dx * dx + dy * dy + dz * dz;
                        knn_insert(bd, bi, &cnt, K, d2, j);
                    }
                }
            }
        }
        double reach = (double)s * csmin;
        if (cnt == K && bd[K - 1] <= reach * reach) break;
    }
    for (int t = 0; t < K; ++t) out[t] = (int32_t)bi[t];
    *h = sqrt(bd[K - 1]);
}

void or_knn_points(const or_sim *S, int32_t inst, int64_t n_q, const double *q, int32_t *ngb,
                   double *h)
{
    for (int64_t t = 0; t < n_q; ++t) knn(S, inst, q + 3 * t, -1, S->p.n_ngb, ngb + t * S->p.n_ngb, h + t);
}

or_sim *or_create(const or_params *p, const double *sigma, const double *eps, int32_t n_inst,
                  const int64_t *inst_off, const double *box, const double *pos, const double *nH,
                  const double *NH, const double *xHI, const double *T)
{
    if (p->n_ngb < 1 || p->n_ngb > 64 || p->n_tc < 3 || p->n_rc < 1 || p->n_rc > 32 ||
        p->n_ec < 1 || p->n_freq < 1 || p->n_em < 1 || p->dt <= 0.0 || n_inst < 1 ||
        p->rr_bin >= p->n_freq || p->max_vip_depth < 1 || p->max_vip_depth > 15 || p->max_hops < 0) {
        set_err("invalid parameters");
        return NULL;
    }
    if ((p->recomb_mode == OR_RR_TRANSPORT || p->recomb_mode == OR_RR_ORIGINAL) && p->rr_bin < 0) {
        set_err("RR transport needs an RR frequency bin");
        return NULL;
    }
    for (int k = 0; k < n_inst; ++k) {
        if (inst_off[k + 1] - inst_off[k] <= p->n_ngb) {
            set_err("every instance needs more than n_ngb particles");
            return NULL;
        }
    }
    or_sim *S = xcalloc(1, sizeof(or_sim));
    S->p = *p;
    S->nf = p->n_freq;
    S->G = p->n_rc * p->n_freq;
    S->n_inst = n_inst;
    S->N = inst_off[n_inst];
    int64_t N = S->N;
    int64_t B = N * S->G;
    S->inst_off = xcalloc((size_t)n_inst + 1, sizeof(int64_t));
    memcpy(S->inst_off, inst_off, sizeof(int64_t) * (n_inst + 1));
    S->box = xcalloc((size_t)n_inst * 6, sizeof(double));
    memcpy(S->box, box, sizeof(double) * 6 * n_inst);
    S->inst_of = xcalloc((size_t)N, sizeof(int32_t));
    for (int k = 0; k < n_inst; ++k)
        for (int64_t i = inst_off[k]; i < inst_off[k + 1]; ++i) S->inst_of[i] = k;
    S->sigma = xcalloc((size_t)S->nf, sizeof(double));
    S->eps = xcalloc((size_t)S->nf, sizeof(double));
    memcpy(S->sigma, sigma, sizeof(double) * S->nf);
    memcpy(S->eps, eps, sizeof(double) * S->nf);
#define DUP(dst, src, n)                            \
    do {                                            \
        dst = xcalloc((size_t)(n), sizeof(double)); \
        memcpy(dst, src, sizeof(double) * (n));     \
    } while (0)
    DUP(S->pos, pos, 3 * N);
    DUP(S->nH, nH, N);
    DUP(S->NH, NH, N);
    DUP(S->xHI, xHI, N);
    DUP(S->T, T, N);
#undef DUP
    S->h = xcalloc((size_t)N, sizeof(double));
    S->ngb = xcalloc((size_t)N * p->n_ngb, sizeof(int32_t));
    S->u_rc = xcalloc((size_t)p->n_rc * 3, sizeof(double));
    S->u_ec = xcalloc((size_t)p->n_ec * 3, sizeof(double));
    S->w_rc = xcalloc((size_t)p->n_rc * 3, sizeof(double));
    or_dirset(p->n_rc, S->u_rc);
    or_dirset(p->n_ec, S->u_ec);
    S->bN = xcalloc((size_t)B, sizeof(double));
    S->bd = xcalloc((size_t)B * 3, sizeof(double));
    S->bc = xcalloc((size_t)B, sizeof(double));
    S->aN = xcalloc((size_t)B, sizeof(double));
    S->aS = xcalloc((size_t)B * 3, sizeof(double));
    S->aC = xcalloc((size_t)B, sizeof(double));
    S->keep = xcalloc((size_t)B, 1);
    S->A = xcalloc((size_t)N * S->nf, sizeof(double));
    S->P = xcalloc((size_t)N * S->nf, sizeof(double));
    S->nrr = xcalloc((size_t)N, sizeof(double));
    S->led = xcalloc((size_t)n_inst * S->nf * 4, sizeof(double));
    S->barrier = xcalloc((size_t)n_inst * 4, sizeof(double));
    build_grid(S);
    /* Neighbour lists (section 2.1), built once: the density field is static. */
    for (int64_t i = 0; i < N; ++i) knn(S, S->inst_of[i], S->pos + 3 * i, i, p->n_ngb, S->ngb + i * p->n_ngb, &S->h[i]);
    return S;
}

void or_destroy(or_sim *S)
{
    if (!S) return;
    free(S->barrier);
    for (int64_t m = 0; m < S->n_emit; ++m) {
        free(S->em[m].pk);
        free(S->em[m].ngb);
    }
    free(S->em);
    free(S->gr);
    free(S->cell_start);
    free(S->cell_idx);
    free(S->inst_off);
    free(S->box);
    free(S->inst_of);
    free(S->sigma);
    free(S->eps);
    free(S->pos);
    free(S->nH);
    free(S->NH);
    free(S->xHI);
    free(S->T);
    free(S->h);
    free(S->ngb);
    free(S->u_rc);
    free(S->u_ec);
    free(S->w_rc);
    free(S->bN);
    free(S->bd);
    free(S->bc);
    free(S->aN);
    free(S->aS);
    free(S->aC);
    free(S->keep);
    free(S->A);
    free(S->P);
    free(S->nrr);
    free(S->led);
    free(S);
}

/* Sources (section 2.1): point sources emit N_EC packets per bin per emission
 * sub-step; photons per packet = rate * dt / (n_em * N_EC).  A plane-parallel
 * front (section 4, footnote on the front) is a regular n x n grid of
 * emitters on the x = lo face of the box, each a packet moving along +x with
 * rate * dt * (cell area) photons per step (reading: it is emitted once per
 * step because it is never rotated). */
int or_add_sources(or_sim *S, int32_t n_src, const int32_t *inst, const int32_t *kind,
                   const double *pos, const double *rate, const int32_t *n_side)
{
    int64_t total = 0;
    for (int s = 0; s < n_src; ++s) {
        if (inst[s] < 0 || inst[s] >= S->n_inst) {
            set_err("source instance out of range");
            return 1;
        }
        if (kind[s] == OR_SRC_POINT)
            total += 1;
        else if (kind[s] == OR_SRC_PLANE_XLO && n_side && n_side[s] >= 1)
            total += (int64_t)n_side[s] * n_side[s];
        else {
            set_err("bad source kind");
            return 1;
        }
    }
    for (int64_t m = 0; m < S->n_emit; ++m) {
        free(S->em[m].pk);
        free(S->em[m].ngb);
    }
    free(S->em);
    S->n_emit = total;
    S->em = xcalloc((size_t)total, sizeof(emitter));
    int64_t m = 0;
    int nf = S->nf;
    for (int s = 0; s < n_src; ++s) {
        int k = inst[s];
        const double *bx = S->box + 6 * k;
        if (kind[s] == OR_SRC_POINT) {
            emitter *e = &S->em[m++];
            e->inst = k;
            e->kind = OR_SRC_POINT;
            e->src = s;
            for (int a = 0; a < 3; ++a) e->pos[a] = pos[3 * s + a];
            e->pk = xcalloc((size_t)nf, sizeof(double));
            for (int nu = 0; nu < nf; ++nu)
                e->pk[nu] = rate[s * nf + nu] * S->p.dt / (double)(S->p.n_em * S->p.n_ec);
        } else {
            int n = n_side[s];
            double dy = (bx[4] - bx[1]) / n, dz = (bx[5] - bx[2]) / n;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    emitter *e = &S->em[m++];
                    e->inst = k;
                    e->kind = OR_SRC_PLANE_XLO;
                    e->src = s;
                    e->pos[0] = bx[0];
                    e->pos[1] = bx[1] + ((double)a + 0.5) * dy;
                    e->pos[2] = bx[2] + ((double)b + 0.5) * dz;
                    e->pk = xcalloc((size_t)nf, sizeof(double));
                    for (int nu = 0; nu < nf; ++nu) e->pk[nu] = rate[s * nf + nu] * S->p.dt * (dy * dz);
                }
        }
    }
    for (int64_t t = 0; t < total; ++t) {
        emitter *e = &S->em[t];
        e->ngb = xcalloc((size_t)S->p.n_ngb, sizeof(int32_t));
        knn(S, e->inst, e->pos, -1, S->p.n_ngb, e->ngb, &e->h);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Transport primitives                                                      */
/* ------------------------------------------------------------------------ */
static int64_t slot_of(const or_sim *S, int64_t i, int nu, int q)
{
    return i * S->G + (int64_t)nu * S->p.n_rc + q;
}

/* Add one arriving packet to the merge accumulators of its reception bin
 * (section 2.1: packets arriving in the same reception cone and frequency bin
 * are merged; photons add, the direction is the luminosity-weighted mean).
 * Reading: clocks merge luminosity-weighted too. */
static void merge_in(or_sim *S, int64_t t, double N, const double d[3], double c)
{
    S->keep[t] = 0;
    S->aN[t] += N;
    S->aS[3 * t + 0] += N * d[0];
    S->aS[3 * t + 1] += N * d[1];
    S->aS[3 * t + 2] += N * d[2];
    S->aC[t] += N * c;
}

/* Split N_in photons over optical depth tau into absorbed N_in (1 - exp(-tau))
 * and transmitted N_in exp(-tau) (section 2.1).  Reading: the smaller of the
 * two parts is evaluated directly and the other is the remainder, so that both
 * keep full relative precision at any tau and their sum is N_in. */
static void attenuate(double N_in, double tau, double *Nabs, double *Nout)
{
    if (tau < 0.6931471805599453) {
        *Nabs = -N_in * expm1(-tau);
        *Nout = N_in - *Nabs;
    } else {
        *Nout = N_in * exp(-tau);
        *Nabs = N_in - *Nout;
    }
}

/* One packet leg onto real particle j (section 2.1): tau = sigma_nu n_HI,j l,
 * N_abs = N_in (1 - exp(-tau)); the rest arrives at j, keeping its direction
 * (reading: the sub-packet keeps the parent's propagation direction), its clock
 * advanced by l / c, and is binned into j's reception cone nearest to d. */
static void leg_to_particle(or_sim *S, int64_t j, int nu, const double d[3], double N_in, double l,
                            double c_prev)
{
    double tau = S->sigma[nu] * S->xHI[j] * S->nH[j] * l;
    double Nabs, Nout;
    attenuate(N_in, tau, &Nabs, &Nout);
    S->A[j * S->nf + nu] += Nabs;
    S->P[j * S->nf + nu] += N_in;
    int r = nearest_dir(S->w_rc, S->p.n_rc, d);
    merge_in(S, slot_of(S, j, nu, r), Nout, d, c_prev + l / C_LIGHT);
}

/* Section 4's artificial barrier: a disk of radius r around c in the plane
 * x = c_x, which removes every photon packet that passes through it.
 * Reading: a packet passes through it when the straight leg it travels, from
 * a to b, meets the disk: the ends are not strictly on one side of the plane,
 * the leg does not lie in the plane, and the point where it meets the plane is
 * within r of c (inclusive).  The removed photons are tallied as removed. */
int or_leg_crosses_disk(const double a[3], const double b[3], const double c[3], double r)
{
    double da = a[0] - c[0], db = b[0] - c[0];
    if ((da > 0.0 && db > 0.0) || (da < 0.0 && db < 0.0)) return 0;
    if (da == db) return 0;
    double t = da / (da - db);
    double py = (a[1] + t * (b[1] - a[1])) - c[1];
    double pz = (a[2] + t * (b[2] - a[2])) - c[2];
    return py * py + pz * pz <= r * r;
}

static int blocked(const or_sim *S, int inst, const double a[3], const double b[3])
{
    const double *bar = S->barrier + 4 * (int64_t)inst;
    return bar[3] > 0.0 && or_leg_crosses_disk(a, b, bar, bar[3]);
}

int or_set_barrier(or_sim *S, int32_t inst, const double center[3], double radius)
{
    if (inst < 0 || inst >= S->n_inst || !(radius >= 0.0)) {
        set_err("bad barrier");
        return 1;
    }
    for (int a = 0; a < 3; ++a) S->barrier[4 * inst + a] = center[a];
    S->barrier[4 * inst + 3] = radius;
    return 0;
}

/* Members of the transmission cone of a packet at position x with direction d
 * among the listed neighbours (in list order).  Returns the count. */
static int cone_members(const or_sim *S, const double x[3], const int32_t *nb, const double d[3],
                        int *mem)
{
    int nc = 0;
    for (int k = 0; k < S->p.n_ngb; ++k) {
        const double *xj = S->pos + 3 * (int64_t)nb[k];
        double v[3] = {xj[0] - x[0], xj[1] - x[1], xj[2] - x[2]};
        if (or_in_cone(v, d, S->p.n_tc)) mem[nc++] = k;
    }
    return nc;
}

/* Cubic-spline SPH kernel shape (Monaghan & Lattanzio 1985, support radius h);
 * the normalisation cancels in the normalised weights used below. */
static double w_spline(double r, double h)
{
    double q = r / h;
    if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) {
        double t = 1.0 - q;
        return 2.0 * t * t * t;
    }
    return 0.0;
}


/* Draw a point uniformly in the unit ball restricted to a cone: rejection from
 * the cube [-1,1]^3.  The cone is either the Voronoi cell ek of the emission
 * directions ecdir (n_ec of them) or the transmission cone around d. */
/* Frame of a transmission cone: its unit axis a = d/|d| and two unit vectors */
/* across it, e1 = (g x a)/|g x a| for the coordinate axis g least aligned    */
/* with a (the first of the smallest |a_k|), and e2 = a x e1.                 */
static void cone_frame(const double d[3], double a[3], double e1[3], double e2[3])
{
    double n = sqrt(dot3(d, d));
    for (int k = 0; k < 3; ++k) a[k] = d[k] / n;
    double ax = fabs(a[0]), ay = fabs(a[1]), az = fabs(a[2]);
    int g = (ax <= ay && ax <= az) ? 0 : (ay <= az ? 1 : 2);
    double c[3];
    /* g x a for the unit vector g */
    if (g == 0) { c[0] = 0.0; c[1] = -a[2]; c[2] = a[1]; }
    else if (g == 1) { c[0] = a[2]; c[1] = 0.0; c[2] = -a[0]; }
    else { c[0] = -a[1]; c[1] = a[0]; c[2] = 0.0; }
    double m = sqrt(dot3(c, c));
    for (int k = 0; k < 3; ++k) e1[k] = c[k] / m;
    e2[0] = a[1] * e1[2] - a[2] * e1[1];
    e2[1] = a[2] * e1[0] - a[0] * e1[2];
    e2[2] = a[0] * e1[1] - a[1] * e1[0];
}

/* A point drawn uniformly in the unit ball intersected with the cone (section */
/* 2.1: the virtual particle lies in the empty cone, within the smoothing      */
/* length).  Reading: rejection sampling, attempt by attempt in order.  A       */
/* transmission cone (axis d, cos theta = 1 - 2/N_TC) draws from the box       */
/* [0, 1] x [-sin theta, sin theta]^2 in its frame, which holds the cone's part */
/* of the ball; an emission cone (a Voronoi cell of the rotated directions)     */
/* draws from the cube [-1, 1]^3.  Either way a point is kept iff it lies in the */
/* ball and passes the cone's own membership test.                            */
static int vip_sample(uint64_t seed, uint32_t tag, uint32_t step, uint32_t ida, uint32_t idb,
                      const double *ecdir, int n_ec, int ek, const double d[3], int n_tc, double p[3])
{
    double a[3], e1[3], e2[3], sn = 0.0;
    if (!ecdir) {
        cone_frame(d, a, e1, e2);
        double c = 1.0 - 2.0 / (double)n_tc;
        sn = sqrt(1.0 - c * c);
    }
    for (uint32_t att = 0; att < VIP_MAX_ATTEMPTS; ++att) {
        double u[4];
        draw4(seed, tag, att, step, ida, idb, u);
        if (ecdir) {
            p[0] = u[0];
            p[1] = u[1];
            p[2] = u[2];
        } else {
            double t = 0.5 * (u[0] + 1.0), x = sn * u[1], y = sn * u[2];
            for (int k = 0; k < 3; ++k) p[k] = t * a[k] + x * e1[k] + y * e2[k];
        }
        if (p[0] * p[0] + p[1] * p[1] + p[2] * p[2] > 1.0) continue;
        if (ecdir) {
            if (nearest_dir(ecdir, n_ec, p) != ek) continue;
        } else if (!or_in_cone(p, d, n_tc)) {
            continue;
        }
        return 1;
    }
    return 0;
}

int or_vip_sample(uint64_t seed, uint32_t tag, uint32_t step, uint32_t ida, uint32_t idb,
                  const double d[3], int32_t n_tc, double p[3])
{
    return vip_sample(seed, tag, step, ida, idb, NULL, 0, 0, d, n_tc, p);
}

typedef struct {
    double x[3];       /* origin of the leg */
    double h;          /* radius of the ball the virtual particle is drawn in */
    double d[3];       /* propagation direction */
    double N, c;       /* photons and clock of the packet */
    int nu;
    int inst;
    const double *ecdir; /* emission directions if the cone is a Voronoi emission cone */
    int ek;              /* its index */
    uint32_t tag, ida, idb_base; /* Philox identity of the draws */
} vip_req;

/* The leg of a packet from x to its virtual particle at xv (section 2.1):
 * the virtual particle's N_ngb nearest particles vn (and its smoothing length
 * hv, the distance to the farthest); its neutral hydrogen density by SPH
 * interpolation, nhi = sum_k w_k x_HI,k n_H,k / sum_k w_k with weights
 * w_k = W(r_k, hv) N_H,k / n_H,k (W the cubic spline, N_H / n_H the particle's
 * volume); the path length l along d; the absorbed Nabs = N (1 - exp(-tau)),
 * tau = sigma_nu nhi l, shared among the neighbours in proportion to w_k
 * (dep[k]), and the rest Nrem.  If every weight vanishes (reading) the
 * neighbours count equally. */
static void vip_leg(const or_sim *S, int inst, const double x[3], const double xv[3], const double d[3], double N,
                    int nu, int32_t *vn, double *hv, double *dep, double *nhi_out, double *l_out, double *Nabs,
                    double *Nrem)
{
    int K = S->p.n_ngb;
    double wk[64];
    knn(S, inst, xv, -1, K, vn, hv);
    double wsum = 0.0, nhi = 0.0;
    for (int k = 0; k < K; ++k) {
        const double *xk = S->pos + 3 * (int64_t)vn[k];
        double dx = xk[0] - xv[0], dy = xk[1] - xv[1], dz = xk[2] - xv[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        wk[k] = w_spline(r, *hv) * (S->NH[vn[k]] / S->nH[vn[k]]);
        wsum += wk[k];
    }
    if (!(wsum > 0.0)) {
        for (int k = 0; k < K; ++k) wk[k] = 1.0;
        wsum = (double)K;
    }
    for (int k = 0; k < K; ++k) nhi += wk[k] * (S->xHI[vn[k]] * S->nH[vn[k]]);
    nhi = nhi / wsum;
    double dd = sqrt(dot3(d, d));
    double l = ((xv[0] - x[0]) * d[0] + (xv[1] - x[1]) * d[1] + (xv[2] - x[2]) * d[2]) / dd;
    double tau = S->sigma[nu] * nhi * l;
    attenuate(N, tau, Nabs, Nrem);
    for (int k = 0; k < K; ++k) dep[k] = *Nabs * wk[k] / wsum;
    *nhi_out = nhi;
    *l_out = l;
}

void or_vip_leg(const or_sim *S, int32_t inst, const double x[3], const double xv[3], const double d[3], double N,
                int32_t nu, int32_t *ngb, double *h, double *dep, double *nhi, double *l, double *Nabs,
                double *Nrem)
{
    vip_leg(S, inst, x, xv, d, N, nu, ngb, h, dep, nhi, l, Nabs, Nrem);
}

/* Virtual particle chain for a packet whose cone holds no neighbour (section
 * 2.1).  Reading: the virtual particle is drawn uniformly in the part of the
 * cone inside the ball of radius h around the origin (rejection from the cube
 * [-1,1]^3); outside the box the packet escapes; otherwise its properties come
 * from SPH interpolation over its own N_ngb neighbours, the leg's absorptions
 * are shared among those neighbours in proportion to W_k N_H,k / n_H,k, and it
 * forwards the rest like a particle.  An empty cone again starts a new
 * virtual particle, up to max_vip_depth; beyond that the packet is removed.
 * Escaped / removed photons are returned through X / R. */
static void vip_chain(or_sim *S, vip_req q, double *X, double *R)
{
    int K = S->p.n_ngb;
    int32_t vn[64];
    int mem[64];
    double wk[64];
    int nf = S->nf;
    const double *bx = S->box + 6 * q.inst;
    for (int depth = 1;; ++depth) {
        S->counters[2]++;
        double p[3] = {0, 0, 0};
        int ok = vip_sample(S->p.seed, q.tag, (uint32_t)S->counters[0], q.ida, q.idb_base | (uint32_t)depth,
                            (q.ecdir && depth == 1) ? q.ecdir : NULL, S->p.n_ec, q.ek, q.d, S->p.n_tc, p);
        if (!ok) {
            *R += q.N;
            return;
        }
        double xv[3] = {q.x[0] + q.h * p[0], q.x[1] + q.h * p[1], q.x[2] + q.h * p[2]};
        if (blocked(S, q.inst, q.x, xv)) {  /* the leg to the virtual particle meets the barrier */
            *R += q.N;
            return;
        }
        for (int a = 0; a < 3; ++a) {
            if (xv[a] < bx[a] || xv[a] > bx[3 + a]) {
                *X += q.N;
                return;
            }
        }
        double hv, nhi, l, Nabs, Nrem;
        vip_leg(S, q.inst, q.x, xv, q.d, q.N, q.nu, vn, &hv, wk, &nhi, &l, &Nabs, &Nrem);
        for (int k = 0; k < K; ++k) S->A[(int64_t)vn[k] * nf + q.nu] += wk[k];
        double dd = sqrt(dot3(q.d, q.d));
        double cv = q.c + l / C_LIGHT;
        int nc = 0;
        for (int k = 0; k < K; ++k) {
            const double *xk = S->pos + 3 * (int64_t)vn[k];
            double v[3] = {xk[0] - xv[0], xk[1] - xv[1], xk[2] - xv[2]};
            if (or_in_cone(v, q.d, S->p.n_tc)) mem[nc++] = k;
        }
        if (nc > 0) {
            double Nin = Nrem / (double)nc;
            for (int t = 0; t < nc; ++t) {
                int64_t j = vn[mem[t]];
                const double *xk = S->pos + 3 * j;
                if (blocked(S, q.inst, xv, xk)) {
                    *R += Nin;
                    continue;
                }
                double v[3] = {xk[0] - xv[0], xk[1] - xv[1], xk[2] - xv[2]};
                double lk = dot3(v, q.d) / dd;
                leg_to_particle(S, j, q.nu, q.d, Nin, lk, cv);
            }
            return;
        }
        if (depth >= S->p.max_vip_depth) {
            *R += Nrem;
            return;
        }
        q.x[0] = xv[0];
        q.x[1] = xv[1];
        q.x[2] = xv[2];
        q.h = hv;
        q.N = Nrem;
        q.c = cv;
    }
}


/* The merged packet from the sums of photons N, of N d and of N clock
 * (section 2.1: direction = luminosity-weighted mean of the parents').  If the
 * weighted directions cancel exactly (reading) the packet takes the axis of
 * its reception cone, fallback_dir. */
static void merged_packet(double N, const double *S3, double NC, const double *fallback_dir,
                          double *oN, double *od, double *oc)
{
    if (N > 0.0) {
        double sx = S3[0], sy = S3[1], sz = S3[2];
        double s2 = sx * sx + sy * sy + sz * sz;
        if (s2 > 0.0) {
            double n = sqrt(s2);
            od[0] = sx / n;
            od[1] = sy / n;
            od[2] = sz / n;
        } else {
            od[0] = fallback_dir[0];
            od[1] = fallback_dir[1];
            od[2] = fallback_dir[2];
        }
        *oN = N;
        *oc = NC / N;
    } else {
        *oN = 0.0;
        od[0] = od[1] = od[2] = 0.0;
        *oc = 0.0;
    }
}

/* Merge n packets given as (N, d, clock) into one, accumulating in list order. */
void or_merge_packets(int32_t n, const double *N, const double *d, const double *c, double *oN,
                      double *od, double *oc)
{
    double aN = 0.0, aS[3] = {0.0, 0.0, 0.0}, aC = 0.0;
    for (int k = 0; k < n; ++k) {
        aN += N[k];
        aS[0] += N[k] * d[3 * k + 0];
        aS[1] += N[k] * d[3 * k + 1];
        aS[2] += N[k] * d[3 * k + 2];
        aC += N[k] * c[k];
    }
    double fb[3] = {1.0, 0.0, 0.0};
    merged_packet(aN, aS, aC, fb, oN, od, oc);
}

/* Convert the merge accumulators back into packets, then deposit packets that
 * fell below the floor (reading: floor_rel * N_H of the holding particle) as
 * absorbed at their particle.  Reading: merging combines the packets that
 * meet in a bin, so a bin that received nothing keeps its packet as it is. */
static void finalize_bins(or_sim *S)
{
    int64_t B = S->N * S->G;
    for (int64_t t = 0; t < B; ++t) {
        if (S->keep[t]) continue;
        int q = (int)(t % S->p.n_rc);
        merged_packet(S->aN[t], S->aS + 3 * t, S->aC[t], S->w_rc + 3 * q, &S->bN[t], S->bd + 3 * t,
                      &S->bc[t]);
    }
    for (int64_t t = 0; t < B; ++t) {
        int64_t i = t / S->G;
        if (S->bN[t] > 0.0 && S->bN[t] < S->p.floor_rel * S->NH[i]) {
            int nu = (int)((t % S->G) / S->p.n_rc);
            S->A[i * S->nf + nu] += S->bN[t];
            S->bN[t] = 0.0;
            S->bd[3 * t] = S->bd[3 * t + 1] = S->bd[3 * t + 2] = 0.0;
            S->bc[t] = 0.0;
        }
    }
}

static void stay(or_sim *S, int64_t t)
{
    double N = S->bN[t];
    S->keep[t] = 1;
    S->aN[t] = N;
    S->aS[3 * t + 0] = N * S->bd[3 * t + 0];
    S->aS[3 * t + 1] = N * S->bd[3 * t + 1];
    S->aS[3 * t + 2] = N * S->bd[3 * t + 2];
    S->aC[t] = N * S->bc[t];
}

static int active(const or_sim *S, int64_t t)
{
    return S->bN[t] > 0.0 && S->bc[t] < S->p.dt;
}

/* Emission at the start of a step (section 2.1): every emission sub-step
 * rotates the N_EC directions at random; reading: the emission cones are the
 * Voronoi cells of the rotated directions, so each source neighbour belongs to
 * the cone of the nearest direction and a packet is shared equally among its
 * cone's members.  Clocks start at the beginning of the step. */
static void emit_sources(or_sim *S, double *Xled, double *Rled)
{
    int nf = S->nf, K = S->p.n_ngb;
    int kc[64], ncount[64], mem[64];
    double ecd[3 * 64];
    for (int64_t m = 0; m < S->n_emit; ++m) {
        emitter *e = &S->em[m];
        int n_sub = e->kind == OR_SRC_POINT ? S->p.n_em : 1;
        for (int sub = 0; sub < n_sub; ++sub) {
            if (e->kind == OR_SRC_POINT) {
                double R[9];
                or_rotation(S->p.seed, TAG_EC, (uint32_t)S->counters[0], (uint32_t)m, (uint32_t)sub, R);
                for (int k = 0; k < S->p.n_ec; ++k) rotate(R, S->u_ec + 3 * k, ecd + 3 * k);
                for (int k = 0; k < S->p.n_ec; ++k) ncount[k] = 0;
                for (int t = 0; t < K; ++t) {
                    const double *xj = S->pos + 3 * (int64_t)e->ngb[t];
                    double v[3] = {xj[0] - e->pos[0], xj[1] - e->pos[1], xj[2] - e->pos[2]};
                    kc[t] = nearest_dir(ecd, S->p.n_ec, v);
                    ncount[kc[t]]++;
                }
                for (int nu = 0; nu < nf; ++nu) {
                    if (!(e->pk[nu] > 0.0)) continue;
                    for (int k = 0; k < S->p.n_ec; ++k) {
                        S->led[((int64_t)e->inst * nf + nu) * 4 + 0] += e->pk[nu];
                        S->counters[3]++;
                    }
                    for (int t = 0; t < K; ++t) {
                        int k = kc[t];
                        int64_t j = e->ngb[t];
                        const double *xj = S->pos + 3 * j;
                        if (blocked(S, e->inst, e->pos, xj)) {
                            Rled[e->inst * nf + nu] += e->pk[nu] / (double)ncount[k];
                            continue;
                        }
                        double v[3] = {xj[0] - e->pos[0], xj[1] - e->pos[1], xj[2] - e->pos[2]};
                        double *dk = ecd + 3 * k;
                        double l = dot3(v, dk) / sqrt(dot3(dk, dk));
                        leg_to_particle(S, j, nu, dk, e->pk[nu] / (double)ncount[k], l, 0.0);
                    }
                    for (int k = 0; k < S->p.n_ec; ++k) {
                        if (ncount[k] > 0) continue;
                        vip_req q;
                        memcpy(q.x, e->pos, sizeof q.x);
                        q.h = e->h;
                        memcpy(q.d, ecd + 3 * k, sizeof q.d);
                        q.N = e->pk[nu];
                        q.c = 0.0;
                        q.nu = nu;
                        q.inst = e->inst;
                        q.ecdir = ecd;
                        q.ek = k;
                        q.tag = TAG_VIP_E;
                        q.ida = (uint32_t)m;
                        q.idb_base = ((uint32_t)sub << 20) | ((uint32_t)k << 4);
                        vip_chain(S, q, &Xled[e->inst * nf + nu], &Rled[e->inst * nf + nu]);
                    }
                }
            } else {
                double d[3] = {1.0, 0.0, 0.0};
                int nc = cone_members(S, e->pos, e->ngb, d, mem);
                for (int nu = 0; nu < nf; ++nu) {
                    if (!(e->pk[nu] > 0.0)) continue;
                    S->led[((int64_t)e->inst * nf + nu) * 4 + 0] += e->pk[nu];
                    S->counters[3]++;
                    if (nc > 0) {
                        for (int t = 0; t < nc; ++t) {
                            int64_t j = e->ngb[mem[t]];
                            const double *xj = S->pos + 3 * j;
                            if (blocked(S, e->inst, e->pos, xj)) {
                                Rled[e->inst * nf + nu] += e->pk[nu] / (double)nc;
                                continue;
                            }
                            double v[3] = {xj[0] - e->pos[0], xj[1] - e->pos[1], xj[2] - e->pos[2]};
                            double l = dot3(v, d) / sqrt(dot3(d, d));
                            leg_to_particle(S, j, nu, d, e->pk[nu] / (double)nc, l, 0.0);
                        }
                    } else {
                        vip_req q;
                        memcpy(q.x, e->pos, sizeof q.x);
                        q.h = e->h;
                        memcpy(q.d, d, sizeof q.d);
                        q.N = e->pk[nu];
                        q.c = 0.0;
                        q.nu = nu;
                        q.inst = e->inst;
                        q.ecdir = NULL;
                        q.ek = 0;
                        q.tag = TAG_VIP_E;
                        q.ida = (uint32_t)m;
                        q.idb_base = 0;
                        vip_chain(S, q, &Xled[e->inst * nf + nu], &Rled[e->inst * nf + nu]);
                    }
                }
            }
        }
    }
}

/* The predecessor scheme of emitting recombination radiation, kept as a
 * reference for the comparison of section 2.2 (the new scheme reuses the
 * reception cones instead).  Every particle is a source of the RR photons of
 * its last chemistry step: like a point source it emits them in N_EC isotropic
 * emission cones on each of the n_em emission sub-steps, with a fresh random
 * rotation per particle and sub-step, into its own neighbours; packets start
 * with clock 0; empty cones become virtual particles.  Reading: its cones are
 * the Voronoi cells of the rotated directions, as for point sources. */
static void emit_rr_original(or_sim *S, uint32_t step, double *Xled, double *Rled)
{
    int nf = S->nf, K = S->p.n_ngb, nu = S->p.rr_bin, nec = S->p.n_ec, nsub = S->p.n_em;
    int kc[64], ncount[64];
    double ecd[3 * 64];
    for (int64_t i = 0; i < S->N; ++i) {
        double nrr = S->nrr[i];
        S->nrr[i] = 0.0;
        if (!(nrr > 0.0)) continue;
        int inst = S->inst_of[i];
        double pk = nrr / (double)(nsub * nec);
        const double *xi = S->pos + 3 * i;
        const int32_t *nb = S->ngb + i * K;
        S->led[((int64_t)inst * nf + nu) * 4 + 0] += nrr;
        for (int sub = 0; sub < nsub; ++sub) {
            double R[9];
            or_rotation(S->p.seed, TAG_RR_EC, step, (uint32_t)i, (uint32_t)sub, R);
            for (int k = 0; k < nec; ++k) {
                rotate(R, S->u_ec + 3 * k, ecd + 3 * k);
                ncount[k] = 0;
            }
            for (int t = 0; t < K; ++t) {
                const double *xj = S->pos + 3 * (int64_t)nb[t];
                double v[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
                kc[t] = nearest_dir(ecd, nec, v);
                ncount[kc[t]]++;
            }
            S->counters[3] += nec;
            for (int t = 0; t < K; ++t) {
                int k = kc[t];
                int64_t j = nb[t];
                const double *xj = S->pos + 3 * j;
                if (blocked(S, inst, xi, xj)) {
                    Rled[inst * nf + nu] += pk / (double)ncount[k];
                    continue;
                }
                double v[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
                double *dk = ecd + 3 * k;
                double l = dot3(v, dk) / sqrt(dot3(dk, dk));
                leg_to_particle(S, j, nu, dk, pk / (double)ncount[k], l, 0.0);
            }
            for (int k = 0; k < nec; ++k) {
                if (ncount[k] > 0) continue;
                vip_req q;
                memcpy(q.x, xi, sizeof q.x);
                q.h = S->h[i];
                memcpy(q.d, ecd + 3 * k, sizeof q.d);
                q.N = pk;
                q.c = 0.0;
                q.nu = nu;
                q.inst = inst;
                q.ecdir = ecd;
                q.ek = k;
                q.tag = TAG_VIP_RR;
                q.ida = (uint32_t)i;
                q.idb_base = ((uint32_t)sub << 20) | ((uint32_t)k << 4);
                vip_chain(S, q, &Xled[inst * nf + nu], &Rled[inst * nf + nu]);
            }
        }
    }
}

/* One RT step followed by the chemistry step (section 2.1) and the emission
 * of recombination radiation into the reception cones (section 2.2).
 * Reading of the order inside a step: (1) clocks carried over from the last
 * step lose dt; (2) the RR photons of the last chemistry step enter the N_RC
 * reception cones of their particle (1/N_RC each, direction = this step's
 * rotated reception direction, clock 0) and merge at once with what is there;
 * (3) sources emit; (4) forward steps until no packet is active; (5)
 * chemistry, which yields the RR photons emitted at the start of the next
 * step. */
static int one_step(or_sim *S)
{
    int nf = S->nf, G = S->G, nrc = S->p.n_rc;
    int64_t N = S->N, B = N * G;
    double dt = S->p.dt;
    uint32_t step = (uint32_t)S->counters[0];
    int hopcap = 0;
    double *Xs = xcalloc((size_t)S->n_inst * nf, sizeof(double));
    double *Rs = xcalloc((size_t)S->n_inst * nf, sizeof(double));

    /* Reception directions of this step (section 2.1: rotated frequently;
     * reading: one random rotation per RT step). */
    or_rotation(S->p.seed, TAG_RC, step, 0, 0, S->rc_rot);
    for (int q = 0; q < nrc; ++q) rotate(S->rc_rot, S->u_rc + 3 * q, S->w_rc + 3 * q);

    memset(S->A, 0, sizeof(double) * N * nf);
    memset(S->P, 0, sizeof(double) * N * nf);

    /* (1) + (2) + (3): everything present stays and merges with new arrivals. */
    for (int64_t t = 0; t < B; ++t) {
        if (S->bN[t] > 0.0) S->bc[t] = S->bc[t] - dt;
        stay(S, t);
    }
    if (S->p.recomb_mode == OR_RR_TRANSPORT) {
        int nu = S->p.rr_bin;
        for (int64_t j = 0; j < N; ++j) {
            if (!(S->nrr[j] > 0.0)) continue;
            double per = S->nrr[j] / (double)nrc;
            for (int q = 0; q < nrc; ++q) merge_in(S, slot_of(S, j, nu, q), per, S->w_rc + 3 * q, 0.0);
            S->led[((int64_t)S->inst_of[j] * nf + nu) * 4 + 0] += S->nrr[j];
            S->nrr[j] = 0.0;
        }
    }
    emit_sources(S, Xs, Rs);
    if (S->p.recomb_mode == OR_RR_ORIGINAL) emit_rr_original(S, step, Xs, Rs);
    finalize_bins(S);

    /* (4) Forward steps (section 2.1): all active packets move at once to the
     * neighbours in their transmission cone; packets move until their clock
     * reaches dt. */
    int *mem = xcalloc(64, sizeof(int));
    int64_t *vips = xcalloc((size_t)B, sizeof(int64_t));
    for (int hop = 1;; ++hop) {
        int64_t n_act = 0;
        for (int64_t t = 0; t < B; ++t) n_act += active(S, t);
        if (n_act == 0) break;
        if (hop > S->p.max_hops) {
            hopcap = 1;
            break;
        }
        S->counters[1]++;
        for (int64_t t = 0; t < B; ++t) {
            if (active(S, t)) {
                S->aN[t] = 0.0;
                S->keep[t] = 0;
                S->aS[3 * t] = S->aS[3 * t + 1] = S->aS[3 * t + 2] = 0.0;
                S->aC[t] = 0.0;
            } else {
                stay(S, t);
            }
        }
        int64_t nv = 0;
        for (int64_t t = 0; t < B; ++t) {
            if (!active(S, t)) continue;
            S->counters[3]++;
            int64_t i = t / G;
            int nu = (int)((t % G) / nrc);
            const double *d = S->bd + 3 * t;
            const int32_t *nb = S->ngb + i * S->p.n_ngb;
            int nc = cone_members(S, S->pos + 3 * i, nb, d, mem);
            if (nc == 0) {
                vips[nv++] = t;
                continue;
            }
            double Nin = S->bN[t] / (double)nc;
            for (int m = 0; m < nc; ++m) {
                int64_t j = nb[mem[m]];
                const double *xi = S->pos + 3 * i, *xj = S->pos + 3 * j;
                if (blocked(S, S->inst_of[i], xi, xj)) {
                    Rs[S->inst_of[i] * nf + nu] += Nin;
                    continue;
                }
                double v[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
                double l = dot3(v, d) / sqrt(dot3(d, d));
                leg_to_particle(S, j, nu, d, Nin, l, S->bc[t]);
            }
        }
        for (int64_t m = 0; m < nv; ++m) {
            int64_t t = vips[m];
            int64_t i = t / G;
            int o = (int)(t % G);
            int nu = o / nrc;
            vip_req q;
            memcpy(q.x, S->pos + 3 * i, sizeof q.x);
            q.h = S->h[i];
            memcpy(q.d, S->bd + 3 * t, sizeof q.d);
            q.N = S->bN[t];
            q.c = S->bc[t];
            q.nu = nu;
            q.inst = S->inst_of[i];
            q.ecdir = NULL;
            q.ek = 0;
            q.tag = TAG_VIP_T;
            q.ida = (uint32_t)i;
            q.idb_base = (((uint32_t)hop & 0xFFFu) << 20) | (((uint32_t)o & 0xFFFFu) << 4);
            vip_chain(S, q, &Xs[q.inst * nf + nu], &Rs[q.inst * nf + nu]);
        }
        finalize_bins(S);
    }
    free(mem);
    free(vips);

    /* (5) Chemistry (section 2.1) and the RR photons it produces (section 2.2). */
    if (!S->p.freeze_chem) {
        for (int64_t j = 0; j < N; ++j) {
            double nrr = 0.0;
            or_chem_one(&S->p, S->eps, S->A + j * nf, S->nH[j], S->NH[j], &S->xHI[j], &S->T[j], &nrr, NULL);
            if (S->p.recomb_mode == OR_RR_TRANSPORT || S->p.recomb_mode == OR_RR_ORIGINAL) S->nrr[j] = nrr;
        }
    } else if (S->p.recomb_mode == OR_RR_TRANSPORT || S->p.recomb_mode == OR_RR_ORIGINAL) {
        /* Frozen ionization state (transport-only runs): the ground-state
         * recombinations of the fixed state over dt still feed the RR bin. */
        double rt[8];
        for (int64_t j = 0; j < N; ++j) {
            or_rates(S->T[j], rt);
            double x = 1.0 - S->xHI[j];
            S->nrr[j] = (rt[0] - rt[1]) * (S->nH[j] * x) * x * S->NH[j] * dt;
        }
    }

    /* Photon ledger (section 2.1: the scheme is explicitly photon-conserving). */
    for (int64_t j = 0; j < N; ++j)
        for (int nu = 0; nu < nf; ++nu) S->led[((int64_t)S->inst_of[j] * nf + nu) * 4 + 1] += S->A[j * nf + nu];
    for (int k = 0; k < S->n_inst; ++k)
        for (int nu = 0; nu < nf; ++nu) {
            S->led[((int64_t)k * nf + nu) * 4 + 2] += Xs[k * nf + nu];
            S->led[((int64_t)k * nf + nu) * 4 + 3] += Rs[k * nf + nu];
        }
    free(Xs);
    free(Rs);
    S->counters[0]++;
    return hopcap;
}

int or_step(or_sim *S, int32_t n_steps)
{
    int rc = 0;
    for (int s = 0; s < n_steps; ++s)
        if (one_step(S)) rc = 4;
    return rc;
}

/* ledger: [n_inst][n_freq][5] = E, A, X, R, F (F = photons still in the bins). */
void or_get_state(const or_sim *S, double *xHI, double *T, double *A, double *P, double *ledger,
                  int64_t *counters)
{
    int64_t N = S->N;
    int nf = S->nf;
    if (xHI) memcpy(xHI, S->xHI, sizeof(double) * N);
    if (T) memcpy(T, S->T, sizeof(double) * N);
    if (A) memcpy(A, S->A, sizeof(double) * N * nf);
    if (P) memcpy(P, S->P, sizeof(double) * N * nf);
    if (ledger) {
        for (int k = 0; k < S->n_inst; ++k)
            for (int nu = 0; nu < nf; ++nu) {
                double *o = ledger + ((int64_t)k * nf + nu) * 5;
                const double *l = S->led + ((int64_t)k * nf + nu) * 4;
                o[0] = l[0];
                o[1] = l[1];
                o[2] = l[2];
                o[3] = l[3];
                double F = 0.0;
                for (int64_t i = S->inst_off[k]; i < S->inst_off[k + 1]; ++i)
                    for (int q = 0; q < S->p.n_rc; ++q) F += S->bN[slot_of(S, i, nu, q)];
                o[4] = F;
            }
    }
    if (counters) memcpy(counters, S->counters, sizeof(S->counters));
}

void or_get_bins(const or_sim *S, double *N, double *d, double *c)
{
    int64_t B = S->N * S->G;
    if (N) memcpy(N, S->bN, sizeof(double) * B);
    if (d) memcpy(d, S->bd, sizeof(double) * B * 3);
    if (c) memcpy(c, S->bc, sizeof(double) * B);
}

void or_get_ngb(const or_sim *S, int32_t *ngb, double *h)
{
    if (ngb) memcpy(ngb, S->ngb, sizeof(int32_t) * S->N * S->p.n_ngb);
    if (h) memcpy(h, S->h, sizeof(double) * S->N);
}

int64_t or_n_emitters(const or_sim *S) { return S->n_emit; }

void or_get_emitter_ngb(const or_sim *S, int32_t *ngb, double *h)
{
    for (int64_t m = 0; m < S->n_emit; ++m) {
        if (ngb) memcpy(ngb + m * S->p.n_ngb, S->em[m].ngb, sizeof(int32_t) * S->p.n_ngb);
        if (h) h[m] = S->em[m].h;
    }
}

void or_get_nrr(const or_sim *S, double *nrr) { memcpy(nrr, S->nrr, sizeof(double) * S->N); }

/* Transmission-cone membership of every active packet of the current bins,
 * as bit k set when neighbour k of the holding particle is in the cone. */
void or_cone_masks(const or_sim *S, uint64_t *mask)
{
    int64_t B = S->N * S->G;
    for (int64_t t = 0; t < B; ++t) {
        mask[t] = 0;
        if (!active(S, t)) continue;
        int64_t i = t / S->G;
        const int32_t *nb = S->ngb + i * S->p.n_ngb;
        for (int k = 0; k < S->p.n_ngb; ++k) {
            const double *xi = S->pos + 3 * i, *xj = S->pos + 3 * (int64_t)nb[k];
            double v[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
            if (or_in_cone(v, S->bd + 3 * t, S->p.n_tc)) mask[t] |= (uint64_t)1 << k;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Intensity profiles (section 3, radial profiles of the Stromgren tests;    */
/* section 4, cylindrical-shell profiles of the shadow test).                */
/* ------------------------------------------------------------------------ */

/* The paper measures the intensity at particle j in bin nu as the photons
 * that passed through j during one RT step divided by that step,
 * I_j = P_j / dt.  Summed over a thin spherical shell around the source this
 * is the number of photons per unit time crossing the sphere of radius r,
 * 4 pi r^2 I(r); the shadow test averages I_j over thin cylindrical shells
 * around the shadow's axis instead, between two planes normal to it.  Bins stay
 * separate, so the source and the diffuse (RR-bin) components are separate
 * columns; both are divided by a normalisation the caller chooses (I_0, the
 * photons emitted per unit time, or a reference shell's value).
 *
 * Shells have width dr = r_max / n_shells; particle j lies in shell
 * floor(r_j / dr) when that is below n_shells, r_j being its distance from
 * center (axis NULL) or from the line through center along axis.  axis may
 * have any nonzero length (it is normalised here); half_height > 0 keeps only
 * particles with |(x_j - center) . u| <= half_height.  mean = 0 sums over the
 * shell, mean = 1 averages over its particles (0 for an empty shell).
 * prof[n_shells * nf] (shell-major), count[n_shells].  Returns 0, or -1 on a
 * bad argument. */
int or_shell_profile(int64_t n, int32_t nf, const double *pos, const double *P, double dt,
                     const double center[3], const double *axis, double half_height, double r_max,
                     int32_t n_shells, int32_t mean, double norm, double *prof, int64_t *count)
{
    if (n < 0 || nf < 1 || n_shells < 1 || !(dt > 0.0) || !(r_max > 0.0) || !(norm > 0.0)) {
        set_err("shell profile: bad argument");
        return -1;
    }
    double u[3] = {0.0, 0.0, 0.0};
    if (axis) {
        double a2 = axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2];
        if (!(a2 > 0.0) || !isfinite(a2)) {
            set_err("shell profile: zero or overflowing axis");
            return -1;
        }
        double a = sqrt(a2);
        for (int k = 0; k < 3; ++k) u[k] = axis[k] / a;
    }
    double dr = r_max / n_shells;
    for (int64_t k = 0; k < (int64_t)n_shells * nf; ++k) prof[k] = 0.0;
    for (int32_t k = 0; k < n_shells; ++k) count[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double *x = pos + 3 * j;
        double d[3] = {x[0] - center[0], x[1] - center[1], x[2] - center[2]};
        double r2;
        if (axis) {
            double t = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
            if (half_height > 0.0 && fabs(t) > half_height) continue;
            double q[3] = {d[0] - t * u[0], d[1] - t * u[1], d[2] - t * u[2]};
            r2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        } else {
            r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        }
        double s = floor(sqrt(r2) / dr);
        if (!(s < (double)n_shells)) continue;
        int32_t k = (int32_t)s;
        count[k] += 1;
        for (int32_t nu = 0; nu < nf; ++nu) prof[(int64_t)k * nf + nu] += P[j * nf + nu] / dt;
    }
    for (int32_t k = 0; k < n_shells; ++k)
        for (int32_t nu = 0; nu < nf; ++nu) {
            double v = prof[(int64_t)k * nf + nu];
            if (mean) v = count[k] > 0 ? v / (double)count[k] : 0.0;
            prof[(int64_t)k * nf + nu] = v / norm;
        }
    return 0;
}
