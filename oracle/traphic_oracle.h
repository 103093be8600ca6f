/*
 * traphic_oracle.h -- plain FP64 CPU oracle of one TRAPHIC radiative-transfer
 * step with recombination-radiation transport (Raicevic, Pawlik, Schaye &
 * Rahmati, "The effect of recombination radiation on the temperature and
 * ionization state of partially ionized gas").
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct
 * reference that the HIP library is checked against.  It shares no code with
 * the HIP library; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.
 *
 * Units are cgs throughout; time in seconds, lengths in cm.
 *
 * Pins (tests/test_oracle_pins.py): Philox known answers; the paper's t_rec,
 * alpha_B/alpha_A, Appendix-B Stromgren distance and mean free path; octant
 * cells of the 8 cube diagonals; Haar statistics of the rotations; cone
 * membership against extended-precision angles, exact integer cases and the
 * 4 pi / N_TC solid angle; uniform virtual-particle sampling (sector centroid);
 * the merge rule; neighbour lists against brute force; 1-D chain attenuation;
 * photon conservation; case-B I-front growth; shell profiles on hand-placed
 * particles and against an independent membership test; the case-B/case-A ratio in the
 * optically thin centre; on-the-spot balance of recombination radiation in
 * optically thick gas; the Riccati closed form of the isothermal chemistry;
 * the light-travel clock (a front stops at the first particle whose projected
 * path reaches c dt and resumes with its clock less dt; clocks advance by the
 * projected path); recombination photons enter the reception cones at clock
 * zero, an equal share per cone; virtual-particle legs (a constant field
 * interpolates to itself, deposits sum to the absorbed photons, the farthest
 * neighbour receives nothing); the section-4 photoheated temperature (soft).
 *
 * parity unpinned: the individual cooling coefficients of or_rates
 * (recombination cooling, collisional ionization and excitation cooling,
 * free-free, Compton; only their combination at the section-4 photoheating
 * equilibrium is pinned, softly, to the paper's 27000 K) and the form of the
 * SPH interpolation weights of virtual particles (W_k N_H,k / n_H,k; only the
 * properties above are pinned).  The paper takes both from predecessor papers
 * it does not reproduce.
 */
#ifndef TRAPHIC_ORACLE_H
#define TRAPHIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* OR_RR_ORIGINAL: RR emitted by every particle in its own N_EC emission cones
 * (the predecessor scheme of section 2.2), a reference for the comparison of
 * the two schemes; the HIP library implements only the reception-cone scheme. */
enum { OR_CASE_B_OTS = 0, OR_CASE_A_NO_RR = 1, OR_RR_TRANSPORT = 2, OR_RR_ORIGINAL = 3 };
enum { OR_SRC_POINT = 0, OR_SRC_PLANE_XLO = 1 };

typedef struct {
    int32_t n_ngb, n_tc, n_rc, n_ec, n_freq, rr_bin;
    int32_t recomb_mode, isothermal, freeze_chem;
    int32_t n_em, max_hops, max_vip_depth;
    double dt, floor_rel, chem_frac;
    uint64_t seed;
} or_params;

typedef struct or_sim or_sim;

/* Returns NULL on invalid input; or_error() then describes it. */
or_sim *or_create(const or_params *p, const double *sigma, const double *eps,
                  int32_t n_inst, const int64_t *inst_off, const double *box,
                  const double *pos, const double *nH, const double *NH,
                  const double *xHI, const double *T);
int or_add_sources(or_sim *S, int32_t n_src, const int32_t *inst, const int32_t *kind,
                   const double *pos, const double *rate, const int32_t *n_side);
/* Runs n steps; returns 0, or 4 when a step stopped at the hop cap. */
int or_step(or_sim *S, int32_t n_steps);
void or_get_state(const or_sim *S, double *xHI, double *T, double *A, double *P,
                  double *ledger, int64_t *counters);
void or_get_bins(const or_sim *S, double *N, double *d, double *c);
void or_get_ngb(const or_sim *S, int32_t *ngb, double *h);
void or_get_emitter_ngb(const or_sim *S, int32_t *ngb, double *h);
int64_t or_n_emitters(const or_sim *S);
void or_cone_masks(const or_sim *S, uint64_t *mask);
void or_get_nrr(const or_sim *S, double *nrr);
void or_destroy(or_sim *S);
const char *or_error(void);

/* Section 4's artificial barrier for instance inst: a disk of the given
 * radius around center in the plane x = center[0]; every packet whose leg
 * meets it is removed (tallied as removed).  radius 0 removes the barrier. */
int or_set_barrier(or_sim *S, int32_t inst, const double center[3], double radius);

/* Primitives exposed for the pin tests. */
int or_leg_crosses_disk(const double a[3], const double b[3], const double c[3], double r);
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_dirset(int32_t n, double *u);
void or_rotation(uint64_t seed, uint32_t tag, uint32_t step, uint32_t a, uint32_t b, double R[9]);
int or_in_cone(const double v[3], const double d[3], int32_t n_tc);
void or_rates(double T, double out[8]);
void or_chem_one(const or_params *p, const double *eps, const double *A, double nH, double NH,
                 double *xHI, double *T, double *nrr, int64_t *nsub);
int or_vip_sample(uint64_t seed, uint32_t tag, uint32_t step, uint32_t ida, uint32_t idb,
                  const double d[3], int32_t n_tc, double p[3]);
void or_merge_packets(int32_t n, const double *N, const double *d, const double *c, double *oN,
                      double *od, double *oc);
void or_knn_points(const or_sim *S, int32_t inst, int64_t n_q, const double *q,
                   int32_t *ngb, double *h);
/* One virtual-particle leg from x to the virtual particle at xv along d
 * (section 2.1): its neighbours ngb[n_ngb] and smoothing length h, the
 * interpolated neutral density nhi, the path length l, the absorbed and
 * remaining photons of a packet of N, and the deposits dep[n_ngb] of the
 * absorbed photons on the neighbours.  Changes nothing in S. */
void or_vip_leg(const or_sim *S, int32_t inst, const double x[3], const double xv[3], const double d[3],
                double N, int32_t nu, int32_t *ngb, double *h, double *dep, double *nhi, double *l,
                double *Nabs, double *Nrem);
/* Intensity profile in spherical or cylindrical shells (sections 3 and 4). */
int or_shell_profile(int64_t n, int32_t nf, const double *pos, const double *P, double dt,
                     const double center[3], const double *axis, double half_height, double r_max,
                     int32_t n_shells, int32_t mean, double norm, double *prof, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif
