/*
 * traphic_rt.h -- C ABI of the MI355X (gfx950) implementation of one TRAPHIC
 * radiative-transfer step on SPH particles with transport of ionizing
 * recombination radiation (RR) in the particles' reception cones, after
 * Raicevic, Pawlik, Schaye & Rahmati, "The effect of recombination radiation
 * on the temperature and ionization state of partially ionized gas".
 *
 * Conventions for every entry point
 *   - Units are cgs: positions in cm, densities in cm^-3, time in s, photon
 *     counts in photons, energies in erg, temperatures in K.
 *   - Array arguments are owned by the caller and only read (inputs) or
 *     written (outputs) during the call.  The arrays of rt_init and
 *     rt_add_sources, and the outputs of rt_get_state, may be host or device
 *     memory (the library asks the runtime which; device inputs are copied to
 *     the host first, since validation reads them there).  Every other array
 *     argument is a host pointer, except passing_dev of
 *     rt_shell_profile_noalloc, which is device memory.  The library copies
 *     inputs to device memory it owns.
 *   - All device work runs on the HIP stream given to rt_init.  rt_step only
 *     enqueues work (it waits on the stream only to decide when a step's
 *     forward steps have finished); rt_get_* synchronise the stream.
 *   - On RT_EINVAL nothing changes.  After RT_EDEVICE only rt_destroy and
 *     rt_last_error are valid.  No C++ exception crosses this interface.
 *   - A context is not thread-safe.
 */
#ifndef TRAPHIC_RT_H
#define TRAPHIC_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx rt_ctx;

typedef enum {
    RT_OK = 0,
    RT_EINVAL = 1,      /* bad argument; the context is unchanged */
    RT_ENOMEM = 2,      /* device allocation failed */
    RT_EDEVICE = 3,     /* a HIP call failed; the context is unusable */
    RT_EHOPCAP = 4,     /* a step stopped at max_hops; unfinished packets stay in flight */
    RT_ENONFINITE = 5,  /* a ledger entry is not finite */
    RT_ESTATE = 6,      /* call out of order (e.g. state blob of the wrong size) */
    RT_EOVERFLOW = 7,   /* the virtual-particle or record buffer overflowed; the packets that
                           found no room left the transport and are counted as removed (the
                           ledger still closes); raise vip_capacity / record_capacity */
    RT_EDRIFT = 8       /* FP32 transport: the photons in flight differ from the ledger's
                           emitted - absorbed - escaped - removed by more than 1e-3 of
                           themselves and more than 1e-5 of the photons emitted (more
                           than rounding), so they were not rescaled (the state stays
                           consistent; the ledger reports the residual) */
} rt_status;

/* Treatment of recombinations (section 2.1 "case B with on-the-spot", "case A";
 * section 2.2 explicit transport of the ground-state recombination photons,
 * emitted into the reception cones; RT_RR_ORIGINAL: the predecessor scheme that
 * section 2.2 compares with, every particle emitting them like a point source
 * in N_EC emission cones rotated per particle and emission sub-step). */
enum { RT_CASE_B_OTS = 0, RT_CASE_A_NO_RR = 1, RT_RR_TRANSPORT = 2, RT_RR_ORIGINAL = 3 };
/* Arithmetic of the packet transport, absorption and merging.  Positions,
 * chemistry and the photon ledger are FP64 in both. */
enum { RT_FP64 = 0, RT_FP32 = 1 };
/* Source kinds: a point source emitting in N_EC randomly rotated directions
 * (section 2.1), or a plane-parallel front entering through the x = lo face
 * of its box as a regular grid of emitters moving along +x (section 4 and its
 * footnote on the front). */
enum { RT_SRC_POINT = 0, RT_SRC_PLANE_XLO = 1 };

typedef struct {
    int32_t n_ngb;         /* SPH neighbours per particle, 1..64 */
    int32_t n_tc;          /* transmission cones: cone solid angle 4 pi / N_TC, >= 3 */
    int32_t n_rc;          /* reception cones per particle and bin: 1, 2, 4, 8, 16 or 32 */
    int32_t n_ec;          /* emission cones of point sources, 1..64 */
    int32_t n_freq;        /* grey frequency bins, 1..15; n_rc * n_freq (the packet slots of a
                              particle) must be a power of two of at most 64, since one
                              wavefront lane holds one slot and a particle's slots share a
                              wavefront (pad with an unused bin if needed) */
    int32_t rr_bin;        /* bin that carries RR photons, or -1 */
    int32_t recomb_mode;   /* RT_CASE_B_OTS, RT_CASE_A_NO_RR, RT_RR_TRANSPORT or RT_RR_ORIGINAL */
    int32_t isothermal;    /* 1: T fixed; 0: photoheating and radiative cooling */
    int32_t freeze_chem;   /* 1: ionization state and T frozen (transport-only runs) */
    int32_t precision;     /* RT_FP64 or RT_FP32 */
    int32_t n_em;          /* emission sub-steps per step (dt / dt_em), >= 1 */
    int32_t max_hops;      /* cap on forward steps per RT step, >= 0 */
    int32_t max_vip_depth; /* virtual particles chained at most this deep, 1..15 */
    int32_t hop_batch;     /* forward steps enqueued between termination checks (0: one
                              more than the previous step needed, then one at a time) */
    double dt;             /* RT and chemistry step, s */
    double floor_rel;      /* packets below floor_rel * N_H of their particle are absorbed there */
    double chem_frac;      /* chemistry sub-step: max relative change of x_HI or T */
    uint64_t seed;         /* key of every random draw (rotations, virtual particles) */
    int64_t vip_capacity;  /* virtual particles per forward step (0: default, the larger of
                              2^16, B/8 and B (1 - 1/n_tc)^n_ngb for B = N n_freq n_rc slots) */
    int64_t record_capacity; /* arrival/deposit records per forward step (0: default, the
                                larger of 2^20 and 4 vip_capacity) */
    /* Optional device allocator (e.g. PyTorch's caching allocator).  NULL: hipMalloc/hipFree.
     * It must return ordinary (coarse-grained) device memory: the kernels add
     * to some arrays with hardware floating-point atomics. */
    void *(*alloc)(void *user, size_t bytes);
    void (*dealloc)(void *user, void *ptr);
    void *alloc_user;
} rt_params;

/* Create a context and build the neighbour lists of the static density field
 * (section 2.1: packets move to neighbours inside the smoothing volume; the
 * density field is static, so the lists are built once).
 *   sigma_nu[n_freq]  grey cross-section per bin, cm^2 (section 2.1 grey approximation)
 *   eps_nu[n_freq]    grey excess energy per photoionization, erg (for the RR bin: k T)
 *   n_inst, inst_off[n_inst+1]  independent problems; particles of instance k
 *                     are inst_off[k] .. inst_off[k+1]-1 (each needs > n_ngb particles)
 *   box[n_inst*6]     lo_x lo_y lo_z hi_x hi_y hi_z of each instance (not periodic)
 *   pos[N*3], n_H[N], N_H[N], x_HI0[N], T0[N]   particle data, N = inst_off[n_inst]
 *   hip_stream        hipStream_t to run on (NULL: the null stream)
 * Errors: RT_EINVAL (parameters, sizes, a particle outside its box), RT_ENOMEM,
 * RT_EDEVICE. */
rt_status rt_init(rt_ctx **out, const rt_params *p, const double *sigma_nu, const double *eps_nu,
                  int32_t n_inst, const int64_t *inst_off, const double *box, const double *pos,
                  const double *n_H, const double *N_H, const double *x_HI0, const double *T0,
                  void *hip_stream);

/* Set the sources (replacing earlier ones).  Section 2.1: a source emits
 * N_EC x N_freq packets per emission sub-step, directions randomly rotated
 * before each emission.
 *   inst[n_src], kind[n_src]   instance and RT_SRC_* kind
 *   pos[n_src*3]               point-source position (ignored for planes; must lie in its box)
 *   rate[n_src*n_freq]         photons/s per bin (point) or photons/s/cm^2 per bin (plane)
 *   n_side[n_src]              plane: emitters per side of the face grid; may be NULL if no planes
 * May be called again between steps (sources switched on during a run).
 * Errors: RT_EINVAL and RT_ENOMEM (the previous sources stay), RT_EDEVICE. */
rt_status rt_add_sources(rt_ctx *ctx, int32_t n_src, const int32_t *inst, const int32_t *kind,
                         const double *pos, const double *rate, const int32_t *n_side);

/* Advance n_steps RT steps, each followed by the chemistry step and the
 * emission of the RR photons into the reception cones (sections 2.1, 2.2).
 * Returns RT_EHOPCAP if a step hit max_hops (the state stays consistent),
 * RT_EOVERFLOW if a work buffer overflowed, RT_ENONFINITE on a non-finite
 * ledger, RT_EDRIFT if the FP32 in-flight rescale was refused, RT_EDEVICE on
 * a HIP failure.  The first of these ends the call after its step; the next
 * call starts afresh. */
rt_status rt_step(rt_ctx *ctx, int32_t n_steps);

/* Copy the state out (synchronises).  Any pointer may be NULL.
 *   x_HI[N], T[N]
 *   absorbed[N*n_freq], passing[N*n_freq]  photons absorbed by / arriving at each
 *                     particle per bin during the last step (section 3 intensity
 *                     diagnostic uses the passing photons)
 *   ledger[n_inst*n_freq*5]  cumulative emitted, absorbed, escaped, removed, and
 *                     photons still in flight (section 2.1: photon conserving)
 *   counters[4]       steps, forward steps, virtual particles, packet updates */
rt_status rt_get_state(rt_ctx *ctx, double *x_HI, double *T, double *absorbed, double *passing,
                       double *ledger, int64_t *counters);

/* Intensity profile of the last step (section 3: radial profiles of the
 * Stromgren tests, split into source and diffuse photons; section 4: profiles
 * of the shadow test in cylindrical shells around the shadow's axis).  The
 * intensity measure at particle j in bin nu is the number of photons that
 * passed through j during the last RT step divided by dt; its sum over a thin
 * spherical shell around the source is the photons per second crossing the
 * sphere of that radius, 4 pi r^2 I(r).  Bins are kept apart, so the RR bin
 * gives the diffuse component.
 *   inst              instance whose particles are binned
 *   passing           NULL: the context's passing photons of the last step;
 *                     else a host array [N*n_freq] (photons) binned instead
 *   center[3]         centre of the spheres, or a point on the cylinder axis (cm)
 *   axis[3]           NULL: spherical shells; else the cylinder axis direction
 *                     (any length whose square is finite and nonzero)
 *   half_height       cylinders: > 0 keeps only particles with
 *                     |(x - center) . axis/|axis|| <= half_height; <= 0: no cut
 *   r_max, n_shells   shells of width r_max / n_shells; particle j lies in shell
 *                     floor(r_j / (r_max / n_shells)) if that is < n_shells
 *                     (r_j: distance from center, or from the axis);
 *                     1 <= n_shells <= 2048, n_shells * n_freq <= 6144
 *   mean              0: sum over the shell; 1: mean over its particles (0 if empty)
 *   norm              > 0; every output is divided by it (e.g. I_0, the source's
 *                     photons per second; 1 for none)
 *   prof[n_shells*n_freq]  out, shell-major, photons/s / norm
 *   count[n_shells]   out, particles per shell (may be NULL)
 * Synchronises the stream.  Errors: RT_EINVAL (nothing written), RT_ENOMEM,
 * RT_EDEVICE. */
rt_status rt_shell_profile(rt_ctx *ctx, int32_t inst, const double *passing, const double *center,
                           const double *axis, double half_height, double r_max, int32_t n_shells,
                           int32_t mean, double norm, double *prof, int64_t *count);

/* rt_shell_profile for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same profile, arguments and limits, with two differences.
 *   passing_dev   NULL: the context's passing photons of the last step; else a
 *                 DEVICE array [N*n_freq] (photons) binned instead (host
 *                 memory is rejected with RT_EINVAL: staging it would allocate)
 *   scratch       the shell histogram lives in a static device array of the
 *                 library, 64 KiB per GPU (6144 sums and 2048 counts: the
 *                 limits above), held until the process ends; it is cleared
 *                 by kernels at every call.
 * No hipMalloc, hipFree or other allocating call is made.  Every call on one
 * GPU uses that GPU's single array: calls that overlap on one GPU (two host
 * threads, or two streams) race and must be serialised by the caller.
 * Synchronises the stream.  Errors: RT_EINVAL (nothing written), RT_EDEVICE. */
rt_status rt_shell_profile_noalloc(rt_ctx *ctx, int32_t inst, const double *passing_dev, const double *center,
                                   const double *axis, double half_height, double r_max, int32_t n_shells,
                                   int32_t mean, double norm, double *prof, int64_t *count);

/* The artificial barrier of the shadow test (section 4): a disk of the given
 * radius (cm) around center[3] in the plane x = center[0], placed in instance
 * inst, which removes every photon packet passing through it.  A packet passes
 * through it when the straight leg it travels (particle to neighbour, emitter
 * to neighbour, to and from a virtual particle) meets the disk: the ends not
 * strictly on one side of the plane, the leg not in the plane, the point where
 * it meets the plane within the radius (inclusive).  Removed photons appear in
 * the ledger as removed.  One disk per instance; radius 0 takes it away (center
 * may then be NULL).  Between steps only; synchronises the stream.  While a
 * disk is set, forward steps run a barrier-aware kernel in the default staging
 * shape (launch configurations then differ in packing only).
 * Errors: RT_EINVAL (nothing changed), RT_EDEVICE. */
rt_status rt_set_barrier(rt_ctx *ctx, int32_t inst, const double *center, double radius);

/* Packet bins [N][n_freq][n_rc] in physical units: photons, unit direction
 * (3 per bin) and clock in s since the start of the last step.  Any pointer may be NULL. */
rt_status rt_get_bins(rt_ctx *ctx, double *N, double *dir, double *clock);

/* Neighbour lists [N][n_ngb] (ascending distance, ties by index) and smoothing
 * lengths h[N] (distance to the n_ngb-th neighbour).  Either may be NULL. */
rt_status rt_get_neighbours(rt_ctx *ctx, int32_t *ngb, double *h);

/* Number of emitters (point sources plus plane-front grid points), and their
 * neighbour lists [n_emit][n_ngb] and h[n_emit]. */
int64_t rt_n_emitters(const rt_ctx *ctx);
rt_status rt_get_emitter_neighbours(rt_ctx *ctx, int32_t *ngb, double *h);

/* Transmission-cone membership of the packets that move in the next forward
 * step: bit k of mask[b] is set when neighbour k of the packet's particle is in
 * the packet's cone; 0 for packets that will not move.  mask[N*n_freq*n_rc]. */
rt_status rt_get_cone_masks(rt_ctx *ctx, uint64_t *mask);

/* Recombination photons waiting to be emitted at the start of the next step, [N]. */
rt_status rt_get_pending_rr(rt_ctx *ctx, double *nrr);

/* Timing of the last rt_step (only when timing is on; synchronises), up to
 * n values: out[0] forward-step kernel total in ms, out[1] its launches,
 * out[2] virtual-particle kernel total ms, out[3] chemistry ms, out[4]
 * emission ms, out[5] ledger ms, out[6] algorithmic bytes the forward-step
 * kernel moved over all its launches (counted on the device from the tiles,
 * edges and packets it handled), out[7] tiles it processed, out[8] bytes of
 * one forward step in the dense model (every slot read and written). */
rt_status rt_set_timing(rt_ctx *ctx, int32_t on);
rt_status rt_get_timing(rt_ctx *ctx, double *out, int32_t n);

/* Launch configuration of the forward steps: incoming edges staged per chunk
 * and (edge, packet) pairs gathered per round, shape % 3 = 0: 256 edges / 128
 * pairs, 1: 128 / 64, 2: 512 / 256 (FP64 gathers half as many pairs, at least
 * 64); shapes 3..5 are 0..2 with up to four tiles (independent wavefronts)
 * per workgroup, which cuts the workgroups a launch dispatches when few tiles
 * have work.  All configurations give identical results.  shape = -1 (the
 * default) lets the library choose among shapes 0..2 (with grids sized from
 * the lists, packing only lowers occupancy once the lists reach their working
 * size): once an RT step needs at least 16 forward steps, the next 3 steps
 * time them (each runs every third forward step, the assignment turning by
 * one from step to step, so that each runs every forward-step index once;
 * forward steps whose list outgrew its grid are not counted) and the fastest
 * per launch is kept; shape = -2 times them on the next 3 steps whatever
 * their size.  RT_EINVAL for another value.  rt_get_hop_shape reports the
 * configuration in use, whether the tuner chose it, and the tuner's mean ms
 * per launch of each (6 doubles, 0 if not timed: always for shapes 3..5);
 * any pointer may be NULL. */
rt_status rt_set_hop_shape(rt_ctx *ctx, int32_t shape);

/* Whole-step graphs (on = 1; default 0): rt_step enqueues each RT step as one
 * captured graph, the steps back to back, with a single host check at the end
 * of the call instead of one per batch of forward steps.  A graph holds at
 * least two forward steps more than the previous step needed, rounded up to a
 * multiple of four; if a step needs more, it
 * halts the queue on the device (every later kernel exits at once) and the
 * call finishes that step one forward step at a time, then goes on.  Used
 * only once a step has run and the launch configuration is settled (not
 * while timing, tuning, or with a fixed hop_batch).  Results are identical
 * either way; the stamps that number forward steps differ.  It is not the
 * default: on the measured workloads it is no faster once its graphs exist
 * and slower while new ones are captured (the fronts' forward-step counts
 * grow).  RT_EINVAL for another value. */
rt_status rt_set_step_graphs(rt_ctx *ctx, int32_t on);
rt_status rt_get_hop_shape(rt_ctx *ctx, int32_t *shape, int32_t *tuned, double *ms_per_launch);

/* Checkpoint: the full dynamic state (bins, ionization state, temperatures,
 * pending RR photons, ledger, counters) as an opaque blob.  rt_get_state_blob
 * with blob == NULL returns the size in *bytes.  rt_set_state_blob restores a
 * blob taken from a context with identical inputs (RT_ESTATE otherwise). */
rt_status rt_get_state_blob(rt_ctx *ctx, void *blob, size_t *bytes);
rt_status rt_set_state_blob(rt_ctx *ctx, const void *blob, size_t bytes);

void rt_destroy(rt_ctx *ctx);
const char *rt_last_error(const rt_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
