// rt_kernels.hpp -- gfx950 kernels of one TRAPHIC RT step with recombination
// radiation.  Layout in HBM:
//   packet bins, slot b = (particle j * n_freq + nu) * n_rc + r:
//     pk[b]  = {dx, dy, dz, N}   (Real4; N in photons / U_inst in FP32 mode)
//     pc[b]  = clock              (s in FP64 mode, units of dt in FP32 mode)
//     cm[b]  = bit k set when neighbour k of j lies in the packet's cone
//     sm[b]  = for receiver slot r of (j, nu): bit p set when packet (j, nu, p)
//              moves this forward step and arrives in reception cone r
//   double-buffered (read one, write the other, swap per forward step).
//   Neighbour lists ngb[j*K+k]; receiver-sorted reverse lists rev_off /
//   rev_ik (sender << 6 | position in the sender's list), sorted by sender,
//   with the edge offsets rev_v; neighbour offsets fwd_v.
#pragma once

#include <cstddef>
#include <type_traits>

#include "rt_device.hpp"

namespace trt {

// counters in device memory, grouped by 64-byte line so that what every
// wavefront reads at the start of a launch never shares a line with what many
// wavefronts write during it
enum : int {
    kCntLine = 8,
    // written once per launch (block 0) or per step
    kCntSteps = 0,
    kCntHops = 1,
    kCntVips = 2,
    kCntUpdates = 3,
    kCntFlags = 4,
    kCntHopsStep = 5,
    kCntRec = 6,
    // lists filled during a launch
    kCntVipCnt0 = 8,   // ViP list fill, ping-pong [8], [9]
    kCntDeep = 10,     // virtual particles of this forward step that landed inside their box
    // nonzero if a packet is active for the next forward step, ping-pong, a line each
    kCntAct0 = 16,     // [16], [24]
    // read at the start of every launch, written rarely
    kCntDone = 32,     // set once a forward step finds no active packet; later launches of the step exit
    kCntSerial = 33,   // stamp of hop 0 of the current RT step (stamps number the forward steps of the run)
    kCntHalt = 34,     // nonzero: every step kernel exits at once (1: a step needs more forward steps
                       // than its graph holds; 2: a step raised an error flag; the forward step
                       // tests the done flag, set with it); cleared by the host
    // per-step tallies
    kCntBytes = 40,    // algorithmic bytes moved by forward steps (for the roofline)
    kCntTiles = 41,    // forward-step tiles processed
    kCntLastHops = 42, // forward steps the last finished RT step ran
    // marked tiles listed for a forward step, ping-pong by its parity: added to
    // by k_tile_list, read by the forward step, cleared by the one before
    kCntTileList = 48,  // [48], [49]
    kCntN = 56
};
// Alignment of the tile-mark array (k_tile_list reads 4096 marks per workgroup).
constexpr long long kTileListChunk = 4096;
enum : long long { kFlagHopCap = 1, kFlagVipOverflow = 2, kFlagRecOverflow = 4, kFlagNonFinite = 8, kFlagDrift = 16 };
// units of the two fixed-point deposit accumulators, relative to the receiving particle's N_H
constexpr double kDepositCoarse = 1.0 / 1073741824.0;         // 2^-30
constexpr double kDepositFine = 1.0 / 4611686018427387904.0;  // 2^-62
constexpr double kDepositFiner = kDepositFine / 4294967296.0;   // 2^-94

template <typename R>
struct alignas(4 * sizeof(R)) Bin4 {
    R x, y, z, n;
};

// Arrival or deposit record of emission and virtual particles (FP64, physical).
struct Rec {
    double nout, dx, dy, dz, clk, nabs, nin;
    unsigned long long key;
    int j;     // receiving particle
    int o;     // slot in the particle (nu * n_rc + r), or -1 - nu for a deposit
};

// A packet whose cone is empty, or an empty emission cone.
struct Vip {
    double x[3], h, d[3], N, c;
    long long xr;              // index into the escaped / removed accumulators
    unsigned long long key;    // base of its records' keys
    int nu, inst;
    int ec;                    // >= 0: Voronoi emission cone (index of its direction set)
    int ek;                    // cone index in that set
    unsigned int tag, ida, idb;
    int xr_emis;               // 1: accumulators of emission virtual particles
};

__device__ inline long long xcd_block(long long b, long long nb) {
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of particles so that neighbours share its L2.
    const long long q = nb / 8, rem = nb % 8;
    const long long x = b % 8, l = b / 8;
    return (x < rem) ? x * (q + 1) + l : rem * (q + 1) + (x - rem) * q + l;
}

// xcd_block for 32-bit counts (shifts and masks only).
__device__ inline unsigned int xcd_block32(unsigned int b, unsigned int nb) {
    const unsigned int q = nb >> 3, rem = nb & 7u;
    const unsigned int x = b & 7u, l = b >> 3;
    return (x < rem) ? x * (q + 1u) + l : rem * (q + 1u) + (x - rem) * q + l;
}

// ------------------------------------------------------------------ set-up --

__global__ void k_fill_i32(int* p, long long n, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double* p, long long n, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_cell_count(long long N, const double* __restrict__ pos, const int* __restrict__ inst_of,
                             const GridInfo* __restrict__ grid, int* __restrict__ cell_of, int* __restrict__ cnt) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const GridInfo g = grid[inst_of[i]];
    int c[3];
    for (int a = 0; a < 3; ++a) {
        int v = static_cast<int>(floor((pos[3 * i + a] - g.lo[a]) / g.cs[a]));
        c[a] = v < 0 ? 0 : (v >= g.nc[a] ? g.nc[a] - 1 : v);
    }
    const long long cell = g.cell0 + (static_cast<long long>(c[0]) * g.nc[1] + c[1]) * g.nc[2] + c[2];
    cell_of[i] = static_cast<int>(cell);
    atomicAdd(&cnt[cell], 1);
}

// Exclusive scan of in[lo, hi) into out[lo, hi), starting from carry0, by one
// workgroup of 1024 threads in sequential chunks; returns the running total.
__device__ inline int scan_range_i32(const int* __restrict__ in, long long lo, long long hi, int carry0,
                                     int* __restrict__ out) {
    __shared__ int part[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = carry0;
    __syncthreads();
    for (long long base = lo; base < hi; base += 1024) {
        const long long i = base + threadIdx.x;
        const int v = i < hi ? in[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < hi) out[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    const int total = carry;
    __syncthreads();
    return total;
}

// Exclusive scan of n ints into out[n+1], one workgroup.
__global__ __launch_bounds__(1024) void k_scan_i32(const int* __restrict__ in, long long n, int* __restrict__ out) {
    const int total = scan_range_i32(in, 0, n, 0, out);
    if (threadIdx.x == 0) out[n] = total;
}

// The same scan over many workgroups, for long arrays (the cells of a finely
// divided grid): workgroup b sums its range [b per, (b + 1) per) (k_scan_sums),
// the sums are scanned by k_scan_i32, and each range is scanned from its offset
// (k_scan_apply).  Integer sums: the result does not depend on the split.
constexpr int kScanBlocks = 1024;
__global__ __launch_bounds__(1024) void k_scan_sums(const int* __restrict__ in, long long n, long long per,
                                                    int* __restrict__ sums) {
    const long long lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    int v = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += 1024) v += in[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ int ws[16];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += ws[w];
        sums[blockIdx.x] = t;
    }
}
__global__ __launch_bounds__(1024) void k_scan_apply(const int* __restrict__ in, long long n, long long per,
                                                     const int* __restrict__ offs, int nb, int* __restrict__ out) {
    const long long lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    (void)scan_range_i32(in, lo, hi, offs[blockIdx.x], out);
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = offs[nb];
}

__global__ void k_cell_fill(long long N, const int* __restrict__ cell_of, const int* __restrict__ start,
                            int* __restrict__ cursor, int* __restrict__ idx) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int c = cell_of[i];
    idx[start[c] + atomicAdd(&cursor[c], 1)] = static_cast<int>(i);
}

// Positions in cell order: entry t is the position of particle cell_idx[t].
__global__ void k_cell_pos(long long N, const int* __restrict__ idx, const double* __restrict__ pos,
                           double* __restrict__ cpos) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= N) return;
    const long long i = idx[t];
    cpos[3 * t] = pos[3 * i];
    cpos[3 * t + 1] = pos[3 * i + 1];
    cpos[3 * t + 2] = pos[3 * i + 2];
}

// k nearest neighbours of points (particles when self >= 0 is their own index).
__global__ __launch_bounds__(128) void k_knn(long long n, const double* __restrict__ qpos, const int* __restrict__ qinst,
                                             int exclude_self, const GridInfo* __restrict__ grid,
                                             const int* __restrict__ cell_start, const int* __restrict__ cell_idx,
                                             const double* __restrict__ pos, int K, int* __restrict__ ngb,
                                             double* __restrict__ h) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double bd[kMaxNgb];
    int bi[kMaxNgb];
    const GridInfo g = grid[qinst[i]];
    h[i] = knn_query(g, cell_start, cell_idx, pos, qpos[3 * i], qpos[3 * i + 1], qpos[3 * i + 2],
                     exclude_self ? static_cast<int>(i) : -1, K, bd, bi);
    for (int k = 0; k < K; ++k) ngb[i * K + k] = bi[k];
}

// The particles' own neighbour lists with the wavefront search (one wavefront
// per particle, four per workgroup): the same lists and smoothing lengths as
// k_knn (the K nearest (d^2, index) pairs are unique), without one thread
// working through every candidate of a dense region alone.
__global__ __launch_bounds__(256) void k_knn_wave(long long n, const double* __restrict__ pos,
                                                  const int* __restrict__ inst_of, const GridInfo* __restrict__ grid,
                                                  const int* __restrict__ cell_start, const int* __restrict__ cell_idx,
                                                  const double* __restrict__ cpos, int K, int* __restrict__ ngb,
                                                  double* __restrict__ h) {
    __shared__ WaveKnn lds[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveKnn& L = lds[wv];
    const long long stride = static_cast<long long>(gridDim.x) * 4;
    for (long long i = static_cast<long long>(blockIdx.x) * 4 + wv; i < n; i += stride) {
        const GridInfo g = grid[inst_of[i]];
        const double qx = pos[3 * i], qy = pos[3 * i + 1], qz = pos[3 * i + 2];
        if (!knn_wave(g, cell_start, cell_idx, cpos, qx, qy, qz, static_cast<int>(i), K, L, lane)) {
            if (lane == 0) {
                knn_query(g, cell_start, cell_idx, pos, qx, qy, qz, static_cast<int>(i), K, L.res_d2, L.res_idx);
                L.kth = L.res_d2[K - 1];
            }
            wave_sync();
        }
        if (lane < K) ngb[i * K + lane] = L.res_idx[lane];
        if (lane == 0) h[i] = sqrt(L.kth);
        wave_sync();  // the wavefront's LDS is reused for its next particle
    }
}

__global__ void k_rev_count(long long nE, const int* __restrict__ ngb, int* __restrict__ cnt) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e < nE) atomicAdd(&cnt[ngb[e]], 1);
}

__global__ void k_rev_fill(long long N, int K, const int* __restrict__ ngb, const int* __restrict__ off,
                           int* __restrict__ cursor, int* __restrict__ src, unsigned char* __restrict__ kpos) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= N * K) return;
    const int j = ngb[e];
    const int t = off[j] + atomicAdd(&cursor[j], 1);
    src[t] = static_cast<int>(e / K);
    kpos[t] = static_cast<unsigned char>(e % K);
}

// Sort each receiver's incoming edges by sender index (deterministic order).
__global__ void k_rev_sort(long long N, const int* __restrict__ off, int* __restrict__ src, unsigned char* __restrict__ kpos) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int a = off[j], b = off[j + 1];
    for (int t = a + 1; t < b; ++t) {
        const int s = src[t];
        const unsigned char k = kpos[t];
        int u = t - 1;
        while (u >= a && src[u] > s) {
            src[u + 1] = src[u];
            kpos[u + 1] = kpos[u];
            --u;
        }
        src[u + 1] = s;
        kpos[u + 1] = k;
    }
}

// Static per-edge data of the forward step: packed reverse edges and offsets.
// FP64: exact offsets.  FP32: receiver-minus-sender offsets in box units and
// unit vectors towards the neighbours, both computed in FP64 and rounded once.
template <typename V4>
__global__ void k_edge_vectors(long long N, int K, const double* __restrict__ pos, const int* __restrict__ ngb,
                               const int* __restrict__ rev_off, const int* __restrict__ rev_src,
                               const unsigned char* __restrict__ rev_pos, const int* __restrict__ inst_of,
                               const double* __restrict__ Linst, unsigned int* __restrict__ rev_ik,
                               V4* __restrict__ rev_v, V4* __restrict__ fwd_v) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    constexpr bool f32 = sizeof(V4) == 16;
    const double Li = f32 ? 1.0 / Linst[inst_of[j]] : 1.0;
    const double xj = pos[3 * j], yj = pos[3 * j + 1], zj = pos[3 * j + 2];
    for (int e = rev_off[j]; e < rev_off[j + 1]; ++e) {
        const long long i = rev_src[e];
        rev_ik[e] = (static_cast<unsigned int>(i) << 6) | rev_pos[e];
        // the forward edge (i, k) learns its receiver-sorted index e in its
        // fourth component (the sender's thread writes only the first three)
        if constexpr (f32)
            fwd_v[i * K + rev_pos[e]].w = __int_as_float(e);
        else
            fwd_v[i * K + rev_pos[e]].w = __longlong_as_double(static_cast<long long>(e));
        const double vx = xj - pos[3 * i], vy = yj - pos[3 * i + 1], vz = zj - pos[3 * i + 2];
        V4 w;
        w.x = vx * Li;
        w.y = vy * Li;
        w.z = vz * Li;
        w.w = 0;
        rev_v[e] = w;
    }
    for (int k = 0; k < K; ++k) {
        const long long n = ngb[j * K + k];
        const double vx = pos[3 * n] - xj, vy = pos[3 * n + 1] - yj, vz = pos[3 * n + 2] - zj;
        V4& w = fwd_v[j * K + k];
        if (f32) {
            const double len = sqrt(vx * vx + vy * vy + vz * vz);
            w.x = vx / len;
            w.y = vy / len;
            w.z = vz / len;
        } else {
            w.x = vx;
            w.y = vy;
            w.z = vz;
        }
    }
}

// Marks the receiver-sorted edges whose leg meets the barrier of their
// instance (section 4): fourth component of the edge vector 1, else 0.
template <typename V4>
__global__ void k_barrier_edges(long long N, const double* __restrict__ pos, const int* __restrict__ rev_off,
                                const unsigned int* __restrict__ rev_ik, const int* __restrict__ inst_of,
                                const double* __restrict__ bar, V4* __restrict__ rev_v) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double xj[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
    const int k = inst_of[j];
    for (int e = rev_off[j]; e < rev_off[j + 1]; ++e) {
        const long long i = rev_ik[e] >> 6;
        const double xi[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        rev_v[e].w = barrier_blocks(bar, k, xi, xj) ? 1 : 0;
    }
}

// ---------------------------------------------------------------- per step --

struct StepBeginArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    const long long* cnt;  // the step number (counted at the step's start) and the halt word
    uint64_t seed;
    int nrc, nec, nsub;
    long long n_emit;
    const double* u_rc;
    const double* u_ec;
    const int* em_kind;
    double* rot;     // [9] rotation of the reception cones + [nrc*3] rotated directions
    float* wrcf;     // float copy of the rotated reception directions
    double* ecd;     // [n_emit][nsub][nec][3] rotated emission directions
};

__global__ void k_step_rotations(StepBeginArgs a) {
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const uint32_t step = static_cast<uint32_t>(a.cnt[kCntSteps] - 1);
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t == 0) {
        double R[9];
        random_rotation(a.seed, kTagRC, step, 0u, 0u, R);
        for (int i = 0; i < 9; ++i) a.rot[i] = R[i];
        for (int q = 0; q < a.nrc; ++q) {
            double w[3];
            rotate3(R, a.u_rc + 3 * q, w);
            for (int c = 0; c < 3; ++c) {
                a.rot[9 + 3 * q + c] = w[c];
                a.wrcf[3 * q + c] = static_cast<float>(w[c]);
            }
        }
    }
    if (t < a.n_emit * a.nsub) {
        const long long m = t / a.nsub;
        const int sub = static_cast<int>(t % a.nsub);
        if (a.em_kind[m] != 0) return;  // plane fronts are not rotated
        double R[9];
        random_rotation(a.seed, kTagEC, step, static_cast<uint32_t>(m), static_cast<uint32_t>(sub), R);
        for (int k = 0; k < a.nec; ++k) rotate3(R, a.u_ec + 3 * k, a.ecd + 3 * ((t * a.nec) + k));
    }
}

struct EmitArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    long long n_emit;
    int K, nf, nrc, nec, nsub, n_em;
    double c2;
    const int* em_kind;
    const int* em_inst;
    const double* em_pos;
    const double* em_pk;   // [n_emit][nf] photons per packet
    const int* em_ngb;
    const double* em_h;
    const double* ecd;
    const double* pos;
    const double* xHI;
    const double* nH;
    const double* sigma;
    const double* wrc;     // rotated reception directions (after the 9 rotation entries)
    Rec* rec;
    int* rec_next;
    int* head;
    long long rec_cap;
    Vip* vip;
    long long vip_cap;
    long long* cnt;
    unsigned long long* xr_fx;  // removed photons of full lists (fixed point, per instance and bin)
    const double* Ufx;
    const double* bar;          // [n_inst][4] barrier disks (section 4)
};

__device__ inline int alloc_records(long long* cnt, int n, long long cap) {
    const long long b = atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[kCntRec]), static_cast<unsigned long long>(n));
    if (b + n > cap) {
        atomicOr(reinterpret_cast<unsigned long long*>(&cnt[kCntFlags]), static_cast<unsigned long long>(kFlagRecOverflow));
        return -1;
    }
    return static_cast<int>(b);
}

__device__ inline void push_record(Rec* rec, int* rec_next, int* head, int idx, const Rec& r) {
    rec[idx] = r;
    rec_next[idx] = atomicExch(&head[r.j], idx);
}

__device__ inline long long push_vip(Vip* vip, long long* cnt, int list, long long cap) {
    const long long b = atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[kCntVipCnt0 + list]), 1ull);
    if (b >= cap) {
        atomicOr(reinterpret_cast<unsigned long long*>(&cnt[kCntFlags]), static_cast<unsigned long long>(kFlagVipOverflow));
        return -1;
    }
    return b;
}

// Adds x >= 0 (in units of an accumulator) to a three-part fixed-point
// accumulator of 64-bit integers in units of 2^-16, 2^-48 and 2^-80: every step
// of the split is exact, integer atomics make the sum independent of the order
// of the adds, and it keeps every bit down to 2^-80 of the unit.  A part beyond
// 2^46 units is refused and flagged (the accumulators could wrap).
__device__ inline void fx_add3(unsigned long long* acc, double x, long long* cnt) {
    if (!(x > 0.0)) return;
    const double xs = x * 65536.0;  // 2^16
    const double c = floor(xs);
    if (!(c < 4503599627370496.0 * 16.0)) {  // 2^56 / 2^10 of headroom per step: 2^46 units
        atomicOr(reinterpret_cast<unsigned long long*>(&cnt[kCntFlags]), static_cast<unsigned long long>(kFlagRecOverflow));
        return;
    }
    const double r1 = (xs - c) * 4294967296.0;  // 2^32
    const double m = floor(r1);
    const long long f = __double2ll_rn((r1 - m) * 4294967296.0);
    if (c > 0.0) atomicAdd(acc, static_cast<unsigned long long>(c));
    if (m > 0.0) atomicAdd(acc + 1, static_cast<unsigned long long>(m));
    if (f) atomicAdd(acc + 2, static_cast<unsigned long long>(f));
}

// fx_add3 for a whole wavefront (every lane calls it; lanes with on = false
// add nothing): the lanes' parts are summed per key across the wavefront
// first (integers: exact, in any order), so each distinct key costs one set
// of atomics instead of one per lane.  key selects acc + 3 key.
__device__ inline void fx_add3_wave(unsigned long long* acc, long long key, double x, bool on, long long* cnt) {
    unsigned long long c = 0, m = 0, f = 0;
    if (on && x > 0.0) {
        const double xs = x * 65536.0;  // 2^16
        const double cd = floor(xs);
        if (!(cd < 4503599627370496.0 * 16.0)) {
            atomicOr(reinterpret_cast<unsigned long long*>(&cnt[kCntFlags]), static_cast<unsigned long long>(kFlagRecOverflow));
        } else {
            const double r1 = (xs - cd) * 4294967296.0;  // 2^32
            const double md = floor(r1);
            c = static_cast<unsigned long long>(cd);
            m = static_cast<unsigned long long>(md);
            f = static_cast<unsigned long long>(__double2ll_rn((r1 - md) * 4294967296.0));
        }
    }
    const int lane = static_cast<int>(threadIdx.x & 63u);
    unsigned long long pend = __ballot((c | m | f) != 0ull);
    while (pend) {
        const int ld = __ffsll(static_cast<long long>(pend)) - 1;
        const long long k = __shfl(key, ld, 64);
        const bool mine = ((pend >> lane) & 1ull) && key == k;
        unsigned long long sc = mine ? c : 0ull, sm = mine ? m : 0ull, sf = mine ? f : 0ull;
        for (int off = 32; off > 0; off >>= 1) {
            sc += __shfl_xor(sc, off, 64);
            sm += __shfl_xor(sm, off, 64);
            sf += __shfl_xor(sf, off, 64);
        }
        if (lane == ld) {
            if (sc) atomicAdd(acc + 3 * k, sc);
            if (sm) atomicAdd(acc + 3 * k + 1, sm);
            if (sf) atomicAdd(acc + 3 * k + 2, sf);
        }
        pend &= ~__ballot(mine);
    }
}

__device__ inline double fx_value3(const unsigned long long* acc) {
    return static_cast<double>(acc[0]) * (1.0 / 65536.0) + static_cast<double>(acc[1]) * (1.0 / 281474976710656.0) +
           static_cast<double>(acc[2]) * (1.0 / 1208925819614629174706176.0);
}

__device__ inline unsigned long long emis_key(long long m, int sub, int nu, int via, int k, int depth, int arr, int kidx) {
    return (static_cast<unsigned long long>(m) << 37) | (static_cast<unsigned long long>(sub) << 25) |
           (static_cast<unsigned long long>(nu) << 21) | (static_cast<unsigned long long>(via) << 20) |
           (static_cast<unsigned long long>(k) << 12) | (static_cast<unsigned long long>(depth) << 8) |
           (static_cast<unsigned long long>(arr) << 7) | static_cast<unsigned long long>(kidx);
}

// Emission (section 2.1): a wavefront per (emitter, sub-step), a lane per
// neighbour (n_ngb <= 64) and per emission cone (n_ec <= 64).  Point sources:
// each neighbour belongs to the Voronoi emission cone of the nearest rotated
// direction; a packet is split equally among its cone's members, counted
// from the lanes' cones (each lane computes its own neighbour's once).  Plane
// fronts: one packet along +x into the transmission cone.
__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const int lane = threadIdx.x & 63;
    const long long ms = blockIdx.x * 4ll + (threadIdx.x >> 6);  // uniform per wavefront
    if (ms >= a.n_emit * a.nsub) return;
    const int sub = static_cast<int>(ms % a.nsub);
    const long long m = ms / a.nsub;
    const int kind = a.em_kind[m];
    if (kind != 0 && sub > 0) return;
    const bool in = lane < a.K;
    const int mem = in ? lane : 0;  // lanes past n_ngb repeat neighbour 0 and are no member
    const double ex = a.em_pos[3 * m], ey = a.em_pos[3 * m + 1], ez = a.em_pos[3 * m + 2];
    const int* nb = a.em_ngb + m * a.K;
    const double* E = a.ecd + 3 * (ms * a.nec);
    const int j = nb[mem];
    const double vx = a.pos[3 * (long long)j] - ex, vy = a.pos[3 * (long long)j + 1] - ey, vz = a.pos[3 * (long long)j + 2] - ez;
    int cone = 0, ncone = 0;
    double dx = 1.0, dy = 0.0, dz = 0.0;
    bool member;
    if (kind == 0) {
        cone = nearest_direction(E, a.nec, vx, vy, vz);
        for (int u = 0; u < a.K; ++u) ncone += __builtin_amdgcn_readlane(cone, u) == cone;
        dx = E[3 * cone];
        dy = E[3 * cone + 1];
        dz = E[3 * cone + 2];
        member = in;
    } else {
        member = in && in_cone(vx, vy, vz, dx, dy, dz, a.c2);
        ncone = __popcll(__ballot(member));
    }
    // members of emission cone `lane` (point sources) or of the one cone (plane fronts)
    int cntk = 0;
    if (kind == 0) {
        for (int u = 0; u < a.K; ++u) cntk += __builtin_amdgcn_readlane(cone, u) == lane;
    } else {
        cntk = ncone;
    }
    const int r = nearest_direction(a.wrc, a.nrc, dx, dy, dz);
    for (int nu = 0; nu < a.nf; ++nu) {
        const double pk = a.em_pk[m * a.nf + nu];
        if (!(pk > 0.0)) continue;
        if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntUpdates]),
                                 static_cast<unsigned long long>(kind == 0 ? a.nec : 1));
        const double xj[3] = {a.pos[3 * (long long)j], a.pos[3 * (long long)j + 1], a.pos[3 * (long long)j + 2]};
        const double xe[3] = {ex, ey, ez};
        if (member && barrier_blocks(a.bar, a.em_inst[m], xe, xj)) {
            // the leg meets the barrier: the member's share is removed
            fx_add3(a.xr_fx + 3 * ((static_cast<long long>(a.em_inst[m]) * a.nf + nu) * 2 + 1),
                    pk / static_cast<double>(ncone) / a.Ufx[a.em_inst[m]], a.cnt);
        } else if (member) {
            const double l = (vx * dx + vy * dy + vz * dz) / sqrt(dx * dx + dy * dy + dz * dz);
            const double nin = pk / static_cast<double>(ncone);
            const double tau = a.sigma[nu] * a.xHI[j] * a.nH[j] * l;
            double nabs, nout;
            attenuate(nin, tau, nabs, nout);
            Rec rc;
            rc.nout = nout;
            rc.dx = dx;
            rc.dy = dy;
            rc.dz = dz;
            rc.clk = 0.0 + l / kCLight;
            rc.nabs = nabs;
            rc.nin = nin;
            rc.key = emis_key(m, sub, nu, 0, 0, 0, 1, mem);
            rc.j = j;
            rc.o = nu * a.nrc + r;
            const int idx = alloc_records(a.cnt, 1, a.rec_cap);
            if (idx >= 0)
                push_record(a.rec, a.rec_next, a.head, idx, rc);
            else  // no room: the member's share leaves the transport as removed
                fx_add3(a.xr_fx + 3 * ((static_cast<long long>(a.em_inst[m]) * a.nf + nu) * 2 + 1), nin / a.Ufx[a.em_inst[m]],
                        a.cnt);
        }
        // Empty cones become virtual particles (lane kk handles cone kk).
        const int nk = kind == 0 ? a.nec : 1;
        if (lane < nk && cntk == 0) {
            const int kk = lane;
            double kx = 1.0, ky = 0.0, kz = 0.0;
            if (kind == 0) {
                kx = E[3 * kk];
                ky = E[3 * kk + 1];
                kz = E[3 * kk + 2];
            }
            const long long v = push_vip(a.vip, a.cnt, 0, a.vip_cap);
            if (v < 0) {  // no room: the empty cone's packet leaves the transport as removed
                fx_add3(a.xr_fx + 3 * ((static_cast<long long>(a.em_inst[m]) * a.nf + nu) * 2 + 1), pk / a.Ufx[a.em_inst[m]],
                        a.cnt);
                continue;
            }
            Vip q;
            q.x[0] = ex;
            q.x[1] = ey;
            q.x[2] = ez;
            q.h = a.em_h[m];
            q.d[0] = kx;
            q.d[1] = ky;
            q.d[2] = kz;
            q.N = pk;
            q.c = 0.0;
            q.nu = nu;
            q.inst = a.em_inst[m];
            q.ec = kind == 0 ? static_cast<int>(ms) : -1;
            q.ek = kk;
            q.tag = kTagVipE;
            q.ida = static_cast<unsigned int>(m);
            q.idb = (static_cast<unsigned int>(sub) << 20) | (static_cast<unsigned int>(kk) << 4);
            q.xr = ((ms * a.nec) + kk) * a.nf + nu;
            q.xr_emis = 1;
            q.key = emis_key(m, sub, nu, 1, kk, 0, 0, 0);
            a.vip[v] = q;
        }
    }
}

// The predecessor scheme of emitting recombination radiation (section 2.2),
// kept to compare with the reception-cone scheme: every particle with RR
// photons from its last chemistry step emits them like a point source, in the
// Voronoi cells of N_EC directions rotated afresh per particle and emission
// sub-step, into its own neighbours (clock 0); empty cells become virtual
// particles.  k_rr_send (thread per particle and sub-step) assigns the
// neighbours to cells and leaves each edge's share and cell on the edge's
// receiver-sorted index; k_rr_recv (thread per particle) attenuates the legs
// arriving at the particle in edge order and sums the packets entering each
// reception cone of the RR bin, which the first forward step merges.
struct RrArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    long long N;
    int K, nf, nrc, nec, nsub, rr_bin;
    uint64_t seed;
    long long m0;               // key index of particle 0's emission (after the sources)
    const double* u_ec;
    const double* pos;
    const double* h;
    const int* ngb;
    const int* inst_of;
    const void* fwd_v;          // fourth component: the edge's receiver-sorted index
    int f32;
    const int* rev_off;
    const unsigned int* rev_ik;
    const double* nrr_prev;
    const double* xHI;
    const double* nH;
    const double* sigma;
    const double* wrc;          // rotated reception directions of this step
    const double* bar;
    double* rr_ecd;             // [N][nsub][nec][3] rotated emission directions
    double* rr_share;           // [edges][nsub] photons per leg (0: none)
    unsigned char* rr_cone;     // [edges][nsub] the leg's cell
    double* rr_pre;             // [N][nrc][6] sums of arrivals: N, N d (3), N c, count
    double* A;
    double* P;
    Vip* vip;
    long long vip_cap;
    unsigned long long* xr_fx;
    const double* Ufx;
    long long* cnt;
};

__global__ __launch_bounds__(64) void k_rr_send(RrArgs a) {
    __shared__ unsigned char kc_s[64 * kMaxNgb];
    __shared__ unsigned char cnt_s[64 * 64];
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const uint32_t step = static_cast<uint32_t>(a.cnt[kCntSteps] - 1);
    const long long t = blockIdx.x * 64ll + threadIdx.x;
    const bool live = t < a.N * a.nsub;
    const long long i = live ? t / a.nsub : 0;
    const int sub = live ? static_cast<int>(t % a.nsub) : 0;
    const double nrr = live ? a.nrr_prev[i] : 0.0;
    const bool emit = live && nrr > 0.0;
    const int nu = a.rr_bin;
    // N_EC packet updates per emitting particle and sub-step, one atomic per wavefront
    const unsigned long long be = __ballot(emit);
    if ((threadIdx.x & 63u) == 0 && be)
        atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntUpdates]),
                  static_cast<unsigned long long>(__popcll(be)) * static_cast<unsigned long long>(a.nec));
    const int inst = a.inst_of[i];
    double removed = 0.0;
    if (emit) {
        const double pk = nrr / static_cast<double>(a.nsub * a.nec);
        double R[9];
        random_rotation(a.seed, kTagRREC, step, static_cast<uint32_t>(i), static_cast<uint32_t>(sub), R);
        double* E = a.rr_ecd + 3 * ((i * a.nsub + sub) * a.nec);
        for (int k = 0; k < a.nec; ++k) rotate3(R, a.u_ec + 3 * k, E + 3 * k);
        unsigned char* kc = kc_s + threadIdx.x * kMaxNgb;
        unsigned char* cn = cnt_s + threadIdx.x * 64;
        for (int k = 0; k < a.nec; ++k) cn[k] = 0;
        const double xi[3] = {a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2]};
        for (int u = 0; u < a.K; ++u) {
            const long long j = a.ngb[i * a.K + u];
            const int k = nearest_direction(E, a.nec, a.pos[3 * j] - xi[0], a.pos[3 * j + 1] - xi[1], a.pos[3 * j + 2] - xi[2]);
            kc[u] = static_cast<unsigned char>(k);
            cn[k] = static_cast<unsigned char>(cn[k] + 1);
        }
        for (int u = 0; u < a.K; ++u) {
            const long long j = a.ngb[i * a.K + u];
            const int k = kc[u];
            long long e;
            if (a.f32)
                e = __float_as_int(static_cast<const float4*>(a.fwd_v)[i * a.K + u].w);
            else
                e = __double_as_longlong(static_cast<const double4*>(a.fwd_v)[i * a.K + u].w);
            double share = pk / static_cast<double>(cn[k]);
            const double xj[3] = {a.pos[3 * j], a.pos[3 * j + 1], a.pos[3 * j + 2]};
            if (barrier_blocks(a.bar, inst, xi, xj)) {  // the leg meets the barrier: removed
                removed += share;
                share = 0.0;
            }
            a.rr_share[e * a.nsub + sub] = share;
            a.rr_cone[e * a.nsub + sub] = static_cast<unsigned char>(k);
        }
        for (int k = 0; k < a.nec; ++k) {
            if (cn[k] != 0) continue;
            const long long v = push_vip(a.vip, a.cnt, 0, a.vip_cap);
            if (v < 0) {  // no room: the empty cell's packet leaves the transport as removed
                removed += pk;
                continue;
            }
            Vip q;
            q.x[0] = xi[0];
            q.x[1] = xi[1];
            q.x[2] = xi[2];
            q.h = a.h[i];
            q.d[0] = E[3 * k];
            q.d[1] = E[3 * k + 1];
            q.d[2] = E[3 * k + 2];
            q.N = pk;
            q.c = 0.0;
            q.nu = nu;
            q.inst = inst;
            q.ec = -2 - static_cast<int>(i * a.nsub + sub);  // its cell: the particle's own direction set
            q.ek = k;
            q.tag = kTagVipRR;
            q.ida = static_cast<unsigned int>(i);
            q.idb = (static_cast<unsigned int>(sub) << 20) | (static_cast<unsigned int>(k) << 4);
            q.xr = 0;
            q.xr_emis = 0;
            q.key = emis_key(a.m0 + i, sub, nu, 1, k, 0, 0, 0);
            a.vip[v] = q;
        }
    }
    fx_add3_wave(a.xr_fx, (static_cast<long long>(inst) * a.nf + nu) * 2 + 1, removed / a.Ufx[inst], removed > 0.0, a.cnt);
}

// thread per particle; each thread's per-cone sums in LDS ([nrc][6] doubles,
// blockDim.x threads per workgroup)
__global__ __launch_bounds__(64) void k_rr_recv(RrArgs a) {
    extern __shared__ __align__(16) unsigned char rr_lds[];
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= a.N) return;
    const int nu = a.rr_bin, nrc = a.nrc;
    double* acc = reinterpret_cast<double*>(rr_lds) + static_cast<size_t>(threadIdx.x) * nrc * 6;
    for (int q = 0; q < 6 * nrc; ++q) acc[q] = 0.0;
    const double xj[3] = {a.pos[3 * j], a.pos[3 * j + 1], a.pos[3 * j + 2]};
    const double sx = a.sigma[nu] * a.xHI[j] * a.nH[j];
    double Aj = 0.0, Pj = 0.0;
    for (int e = a.rev_off[j]; e < a.rev_off[j + 1]; ++e) {
        const long long i = a.rev_ik[e] >> 6;
        if (!(a.nrr_prev[i] > 0.0)) continue;
        const double vx = xj[0] - a.pos[3 * i], vy = xj[1] - a.pos[3 * i + 1], vz = xj[2] - a.pos[3 * i + 2];
        for (int sub = 0; sub < a.nsub; ++sub) {
            const double share = a.rr_share[static_cast<long long>(e) * a.nsub + sub];
            if (!(share > 0.0)) continue;
            const int k = a.rr_cone[static_cast<long long>(e) * a.nsub + sub];
            const double* d = a.rr_ecd + 3 * ((i * a.nsub + sub) * a.nec + k);
            const double l = (vx * d[0] + vy * d[1] + vz * d[2]) / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double nabs, nout;
            attenuate(share, sx * l, nabs, nout);
            Aj += nabs;
            Pj += share;
            double* s6 = acc + 6 * nearest_direction(a.wrc, nrc, d[0], d[1], d[2]);
            s6[0] += nout;
            s6[1] += nout * d[0];
            s6[2] += nout * d[1];
            s6[3] += nout * d[2];
            s6[4] += nout * (0.0 + l / kCLight);
            s6[5] += 1.0;
        }
    }
    double* pr = a.rr_pre + 6 * j * nrc;
    for (int q = 0; q < 6 * nrc; ++q) pr[q] = acc[q];
    if (Pj > 0.0) {
        a.A[j * a.nf + nu] += Aj;
        a.P[j * a.nf + nu] += Pj;
    }
}

// One workgroup (256 threads) lists the marked tiles of mark chunk `chunk`
// (kTileListChunk marks, 16 consecutive per thread, read as four 16-byte
// vectors): a workgroup prefix sum orders them and one atomic on *count
// places them.  Every thread of the workgroup must call it.
__device__ __forceinline__ void list_marked_chunk(const int* __restrict__ hot, long long ntiles, int stamp, long long chunk,
                                                  const int* __restrict__ rev_off, long long N, int T,
                                                  int4* __restrict__ tlist, long long* count) {
    const long long t0 = chunk * kTileListChunk + threadIdx.x * 16ll;
    const int4* h4 = reinterpret_cast<const int4*>(hot + t0);  // the mark array is padded to whole chunks
    unsigned int bits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int4 v = h4[q];
        bits |= (v.x == stamp ? 1u : 0u) << (4 * q);
        bits |= (v.y == stamp ? 1u : 0u) << (4 * q + 1);
        bits |= (v.z == stamp ? 1u : 0u) << (4 * q + 2);
        bits |= (v.w == stamp ? 1u : 0u) << (4 * q + 3);
    }
    if (t0 + 16 > ntiles) bits &= t0 >= ntiles ? 0u : ((1u << (ntiles - t0)) - 1u);
    const int mine = __popc(bits);
    // exclusive prefix over the workgroup, in thread (= tile) order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    __shared__ int wtot[4];
    __shared__ long long base;
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < 4; ++w) {
        before += w < wv ? wtot[w] : 0;
        total += wtot[w];
    }
    if (threadIdx.x == 0)
        base = total ? static_cast<long long>(atomicAdd(reinterpret_cast<unsigned long long*>(count),
                                                        static_cast<unsigned long long>(total)))
                     : 0ll;
    __syncthreads();
    long long at = base + before + incl - mine;
    __syncthreads();  // wtot and base are free for the workgroup's next chunk
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        const long long t = t0 + b, j0 = t * T, j1 = (j0 + T < N) ? j0 + T : N;
        tlist[at++] = make_int4(static_cast<int>(t), rev_off[j0], rev_off[j1], 0);
    }
}

struct VipArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    const double* rr_ecd;  // direction sets of the predecessor RR scheme (virtual particles with ec <= -2)
    int hop, hop0, max_hops, K, nf, nrc, nec, max_depth;
    long long* dep;  // [N*nf][3] deposited photons of virtual-particle legs, fixed point
    uint64_t seed;
    double c2;
    const Vip* list;
    long long vip_cap;
    const double* box;
    const GridInfo* grid;
    const int* cell_start;
    const int* cell_idx;
    const double* cell_pos;
    const double* pos;
    const double* xHI;
    const double* nH;
    const double* NH;
    const double* sigma;
    const double* wrc;
    const double* ecd;
    unsigned long long* xr_fx;  // [n_inst][nf][2][3] escaped, removed photons of transport
                                // virtual particles this step, fixed point (fx_add3)
    const double* Ufx;          // [n_inst] unit of those accumulators: the mean N_H
    const double* bar;          // [n_inst][4] barrier disks (section 4)
    double* exs;     // escaped per emission packet
    double* ers;     // removed per emission packet
    Rec* rec;
    int* rec_next;
    int* head;
    long long rec_cap;
    int* hot;        // marks of this forward step's tiles (deliveries of the previous one, records)
    int lgT;
    // hop > 0: k_vip_sample lists the tiles the previous forward step marked,
    // and k_vip_chain appends those it marks first (no separate list launch)
    int list_here;
    int4* tlist;
    const int* rev_off;
    long long N, ntiles, nchunks;
    int T;
    Vip* deep;       // virtual particles that landed inside their box, with their points
    double* deep_x;
    long long* cnt;
    int act_rd, act_wr, list_rd, list_wr;
};

// Virtual particles (section 2.1).  The particle is drawn uniformly in the
// cone inside the ball of radius h around the origin (rejection from the cube
// [-1,1]^3, Philox draws numbered by attempt, the lowest accepted attempt
// wins); outside the box the packet escapes; otherwise it takes
// SPH-interpolated properties from its own N_ngb neighbours, the leg's
// absorptions go to those neighbours in proportion to W_k N_H,k / n_H,k, and
// it forwards the rest into its own transmission cone (chaining up to
// max_depth).  k_vip_sample draws the first point of every chain, one lane
// each, and settles those that escape; the rest go on to k_vip_chain.

// A group of kVipLanes lanes draws attempts kVipLanes at a time (attempt
// round*kVipLanes + sub-lane); the lowest accepted attempt wins, as if drawn
// one by one.  Every lane of the group returns the point.  False if no attempt
// is accepted.
constexpr int kVipLanes = 4;

__device__ inline bool vip_draw_group(const VipArgs& a, uint32_t step, const Vip& q, bool live, int depth, int sub,
                                      int gshift, double p[3]) {
    // depth 1 of an emission cone: its Voronoi cell (a source's set, or with
    // ec <= -2 a particle's set of the predecessor RR scheme)
    const double* ecs = depth != 1 ? nullptr
                        : q.ec >= 0 ? a.ecd + 3 * (static_cast<long long>(q.ec) * a.nec)
                        : q.ec <= -2 ? a.rr_ecd + 3 * ((-2ll - q.ec) * a.nec)
                                     : nullptr;
    const ConeFrame fr = cone_frame(q.d, a.c2);
    const unsigned long long gm = (kVipLanes >= 64 ? ~0ull : ((1ull << kVipLanes) - 1ull)) << gshift;
    bool done = !live;
    bool found = false;
    for (uint32_t base = 0; base < kVipAttempts; base += kVipLanes) {
        bool ok = false;
        double u[4] = {0.0, 0.0, 0.0, 0.0};
        if (!done) {
            uniforms4(a.seed, q.tag, base + static_cast<uint32_t>(sub), step, q.ida, q.idb | static_cast<uint32_t>(depth), u);
            if (!ecs) {
                double pc[3];
                cone_point(fr, u, pc);
                u[0] = pc[0];
                u[1] = pc[1];
                u[2] = pc[2];
            }
            ok = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= 1.0;
            if (ok) ok = ecs ? nearest_direction(ecs, a.nec, u[0], u[1], u[2]) == q.ek
                             : in_cone(u[0], u[1], u[2], q.d[0], q.d[1], q.d[2], a.c2);
        }
        const unsigned long long b = __ballot(ok) & gm;
        if (b && !done) {
            const int f = __ffsll(static_cast<long long>(b)) - 1;  // lowest attempt of the group
            p[0] = __shfl(u[0], f, 64);
            p[1] = __shfl(u[1], f, 64);
            p[2] = __shfl(u[2], f, 64);
            found = true;
            done = true;
        }
        if (__ballot(!done) == 0) break;
    }
    return found;
}

// A virtual particle's packet leaves the transport: escaped (what = 0, its
// point lies outside the box) or removed (what = 1, no point found, or the
// chain too deep).  Emission cones keep per-packet sums (k_emit_tally); transport
// packets add to their instance's fixed-point accumulators.
__device__ inline void vip_settle(const VipArgs& a, const Vip& q, int what, double n) {
    if (q.xr_emis) {
        (what ? a.ers : a.exs)[q.xr] += n;
    } else {
        fx_add3(a.xr_fx + 3 * ((static_cast<long long>(q.inst) * a.nf + q.nu) * 2 + what), n / a.Ufx[q.inst], a.cnt);
    }
}

__global__ __launch_bounds__(256) void k_vip_sample(VipArgs a) {
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    // after hop 0 the first a.nchunks workgroups list the marked tiles (one
    // chunk of marks each) and the others take the virtual particles, so the
    // two run side by side
    const long long nlist = a.list_here ? a.nchunks : 0;
    const long long vblk = static_cast<long long>(blockIdx.x) - nlist;
    const long long gid = vblk * 256LL + threadIdx.x;
    if (!a.hop0) {
        // Once one forward step has found nothing to move, every later launch
        // of this step must exit: the ping-pong counters it would read are stale.
        if (a.cnt[kCntDone] != 0 || a.cnt[kCntAct0 + kCntLine * a.act_rd] == 0 || a.hop > a.max_hops) {
            if (gid == 0) a.cnt[kCntDone] = 1;
            return;
        }
    }
    if (vblk < 0) {
        // the tiles the previous forward step marked for this one
        list_marked_chunk(a.hot, a.ntiles, static_cast<int>(a.cnt[kCntSerial]) + a.hop, blockIdx.x, a.rev_off, a.N, a.T,
                          a.tlist, &a.cnt[kCntTileList + (a.hop & 1)]);
        return;
    }
    long long n = a.cnt[kCntVipCnt0 + a.list_rd];
    if (n > a.vip_cap) n = a.vip_cap;
    if (gid == 0) {
        a.cnt[kCntAct0 + kCntLine * a.act_wr] = 0;
        a.cnt[kCntVipCnt0 + a.list_wr] = 0;
        a.cnt[kCntVips] += n;  // the first leg of every chain
    }
    const uint32_t step = static_cast<uint32_t>(a.cnt[kCntSteps] - 1);  // the step counter counts this step
    const int lane = threadIdx.x & 63;
    const int sub = lane % kVipLanes;
    const int gshift = lane - sub;
    const long long groups = (static_cast<long long>(gridDim.x) - nlist) * (256LL / kVipLanes);
    const long long g0 = gid / kVipLanes;
    // a uniform trip count per wavefront: its groups stay in step
    const long long wbase = (gid - lane) / kVipLanes;
    for (long long vb = wbase; vb < n; vb += groups) {
        const long long v = vb + (g0 - wbase);
        const bool live = v < n;
        Vip q = {};
        if (live) q = a.list[v];
        double p[3] = {0.0, 0.0, 0.0};
        const bool found = vip_draw_group(a, step, q, live, 1, sub, gshift, p);
        bool inside = false;
        double xv[3] = {0.0, 0.0, 0.0};
        int what = -1;  // 0 escaped, 1 removed (no point found)
        if (live && sub == 0) {
            const double* bx = a.box + 6 * q.inst;
            if (!found) {
                what = 1;
            } else {
                xv[0] = q.x[0] + q.h * p[0];
                xv[1] = q.x[1] + q.h * p[1];
                xv[2] = q.x[2] + q.h * p[2];
                if (barrier_blocks(a.bar, q.inst, q.x, xv))
                    what = 1;  // the leg to the virtual particle meets the barrier
                else if (xv[0] < bx[0] || xv[0] > bx[3] || xv[1] < bx[1] || xv[1] > bx[4] || xv[2] < bx[2] || xv[2] > bx[5])
                    what = 0;
                else
                    inside = true;
            }
            if (what >= 0 && q.xr_emis) (what ? a.ers : a.exs)[q.xr] += q.N;
        }
        // transport packets: one set of atomics per (instance, bin, kind) in the wavefront
        const bool tr = what >= 0 && !q.xr_emis;
        fx_add3_wave(a.xr_fx, tr ? (static_cast<long long>(q.inst) * a.nf + q.nu) * 2 + what : 0, tr ? q.N / a.Ufx[q.inst] : 0.0,
                     tr, a.cnt);
        // append the inside ones, one atomic per wavefront
        const unsigned long long b = __ballot(inside);
        if (b) {
            long long base = 0;
            if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntDeep]), static_cast<unsigned long long>(__popcll(b)));
            base = __shfl(base, 0, 64);
            if (inside) {
                const long long d = base + __popcll(b & ((1ull << lane) - 1ull));
                if (d < a.vip_cap) {
                    a.deep[d] = q;
                    a.deep_x[3 * d] = xv[0];
                    a.deep_x[3 * d + 1] = xv[1];
                    a.deep_x[3 * d + 2] = xv[2];
                } else {
                    // no room to follow it: its photons leave the transport as removed
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagVipOverflow));
                    vip_settle(a, q, 1, q.N);
                }
            }
        }
    }
}

// One wavefront per chain that landed inside its box: its neighbours (one
// lane each), the leg, and further legs if the cone is empty again (their
// points drawn by the whole wavefront, 64 attempts at a time).
__global__ __launch_bounds__(256) void k_vip_chain(VipArgs a) {
    __shared__ WaveKnn lds[4];
    __shared__ double rcd[96];  // the step's reception-cone directions
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    if (threadIdx.x < 3 * a.nrc) rcd[threadIdx.x] = a.wrc[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long long gw = blockIdx.x * 4LL + wv;
    const long long nw = gridDim.x * 4LL;
    long long n = a.cnt[kCntDeep];
    if (n > a.vip_cap) n = a.vip_cap;
    const uint32_t step = static_cast<uint32_t>(a.cnt[kCntSteps] - 1);
    const int stamp = static_cast<int>(a.cnt[kCntSerial]) + a.hop;
    WaveKnn& L = lds[wv];
    const int K = a.K;
    for (long long v = gw; v < n; v += nw) {
        Vip q = a.deep[v];
        const double* bx = a.box + 6 * q.inst;
        const GridInfo g = a.grid[q.inst];
        double xv[3] = {a.deep_x[3 * v], a.deep_x[3 * v + 1], a.deep_x[3 * v + 2]};
        for (int depth = 1;; ++depth) {
            if (depth > 1) {
                if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntVips]), 1ull);
                double p0 = 0.0, p1 = 0.0, p2 = 0.0;
                bool found = false;
                const ConeFrame fr = cone_frame(q.d, a.c2);
                for (uint32_t base = 0; base < kVipAttempts; base += 64) {
                    double u[4];
                    uniforms4(a.seed, q.tag, base + lane, step, q.ida, q.idb | static_cast<uint32_t>(depth), u);
                    double pc[3];
                    cone_point(fr, u, pc);
                    u[0] = pc[0];
                    u[1] = pc[1];
                    u[2] = pc[2];
                    bool ok = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= 1.0;
                    if (ok) ok = in_cone(u[0], u[1], u[2], q.d[0], q.d[1], q.d[2], a.c2);
                    const unsigned long long b = __ballot(ok);
                    if (b) {
                        const int f = __ffsll(static_cast<long long>(b)) - 1;
                        p0 = __shfl(u[0], f, 64);
                        p1 = __shfl(u[1], f, 64);
                        p2 = __shfl(u[2], f, 64);
                        found = true;
                        break;
                    }
                }
                if (!found) {
                    if (lane == 0) vip_settle(a, q, 1, q.N);
                    break;
                }
                xv[0] = q.x[0] + q.h * p0;
                xv[1] = q.x[1] + q.h * p1;
                xv[2] = q.x[2] + q.h * p2;
                if (barrier_blocks(a.bar, q.inst, q.x, xv)) {
                    if (lane == 0) vip_settle(a, q, 1, q.N);
                    break;
                }
                if (xv[0] < bx[0] || xv[0] > bx[3] || xv[1] < bx[1] || xv[1] > bx[4] || xv[2] < bx[2] || xv[2] > bx[5]) {
                    if (lane == 0) vip_settle(a, q, 0, q.N);
                    break;
                }
            }
            if (!knn_wave(g, a.cell_start, a.cell_idx, a.cell_pos, xv[0], xv[1], xv[2], -1, K, L, lane)) {
                // candidate buffer overflow (very clustered cells): serial query on one lane
                if (lane == 0) {
                    double bd[kMaxNgb];
                    int bi[kMaxNgb];
                    knn_query(g, a.cell_start, a.cell_idx, a.pos, xv[0], xv[1], xv[2], -1, K, bd, bi);
                    for (int k = 0; k < K; ++k) {
                        L.res_d2[k] = bd[k];
                        L.res_idx[k] = bi[k];
                    }
                    L.kth = bd[K - 1];
                }
                wave_sync();
            }
            const bool nbl = lane < K;
            const long long jk = nbl ? L.res_idx[lane] : 0;
            const double d2k = nbl ? L.res_d2[lane] : 0.0;
            const double hv = sqrt(L.kth);
            wave_sync();
            // everything the leg needs of the neighbour, loaded together
            const double NHk = a.NH[jk], nHk = a.nH[jk], xHk = a.xHI[jk];
            const double pxk = a.pos[3 * jk], pyk = a.pos[3 * jk + 1], pzk = a.pos[3 * jk + 2];
            double w = nbl ? spline_shape(sqrt(d2k), hv) * (NHk / nHk) : 0.0;
            double wsum = wave_sum(w);
            if (!(wsum > 0.0)) {
                w = nbl ? 1.0 : 0.0;
                wsum = static_cast<double>(K);
            }
            const double nhi = wave_sum(nbl ? w * (xHk * nHk) : 0.0) / wsum;
            const double dd = sqrt(q.d[0] * q.d[0] + q.d[1] * q.d[1] + q.d[2] * q.d[2]);
            const double l = ((xv[0] - q.x[0]) * q.d[0] + (xv[1] - q.x[1]) * q.d[1] + (xv[2] - q.x[2]) * q.d[2]) / dd;
            const double tau = a.sigma[q.nu] * nhi * l;
            double nabs, nrem;
            attenuate(q.N, tau, nabs, nrem);
            // deposits of the leg's absorptions to the neighbours, as integers
            // (order-independent, deterministic sums) in units of N_H,k 2^-30,
            // 2^-62 and 2^-94: every step of the split is exact, so the three
            // parts hold all the bits of the deposit down to 2^-94 N_H,k (a bin
            // with photons far below N_H keeps its relative precision)
            if (nbl) {
                const double x = (nabs * w / wsum) / NHk * 1073741824.0;  // 2^30
                if (x > 0.0) {
                    double cpart = floor(x);
                    if (!(cpart < 9.0e18)) {
                        cpart = 9.0e18;
                        atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagRecOverflow));
                    }
                    const double r1 = (x - cpart) * 4294967296.0;  // 2^32
                    const double mpart = floor(r1);
                    const long long ic = static_cast<long long>(cpart);
                    const long long im = static_cast<long long>(mpart);
                    const long long ifn = __double2ll_rn((r1 - mpart) * 4294967296.0);
                    unsigned long long* d = reinterpret_cast<unsigned long long*>(&a.dep[3 * (jk * a.nf + q.nu)]);
                    if (ic) atomicAdd(d, static_cast<unsigned long long>(ic));
                    if (im) atomicAdd(d + 1, static_cast<unsigned long long>(im));
                    if (ifn) atomicAdd(d + 2, static_cast<unsigned long long>(ifn));
                }
            }
            const double cv = q.c + l / kCLight;
            double vx = 0.0, vy = 0.0, vz = 0.0;
            bool member = false;
            if (nbl) {
                vx = pxk - xv[0];
                vy = pyk - xv[1];
                vz = pzk - xv[2];
                member = in_cone(vx, vy, vz, q.d[0], q.d[1], q.d[2], a.c2);
            }
            const unsigned long long bm = __ballot(member);
            const int nc = __popcll(bm);
            if (nc > 0) {
                const int r = nearest_direction(static_cast<const double*>(rcd), a.nrc, q.d[0], q.d[1], q.d[2]);
                const double nin = nrem / static_cast<double>(nc);
                int idx1 = 0;
                if (lane == 0) idx1 = alloc_records(a.cnt, nc, a.rec_cap);
                idx1 = __shfl(idx1, 0, 64);
                if (idx1 < 0 && lane == 0) vip_settle(a, q, 1, nrem);  // no room: removed
                // members whose leg meets the barrier: their shares are removed
                const double xk[3] = {pxk, pyk, pzk};
                const bool cut = member && idx1 >= 0 && barrier_blocks(a.bar, q.inst, xv, xk);
                if (q.xr_emis) {
                    const unsigned long long bc = __ballot(cut);
                    if (bc && lane == 0) a.ers[q.xr] += nin * static_cast<double>(__popcll(bc));
                } else {
                    fx_add3_wave(a.xr_fx, (static_cast<long long>(q.inst) * a.nf + q.nu) * 2 + 1,
                                 cut ? nin / a.Ufx[q.inst] : 0.0, cut, a.cnt);
                }
                if (member && idx1 >= 0 && !cut) {
                    const int w8 = __popcll(bm & ((1ull << lane) - 1ull));
                    const double lk = (vx * q.d[0] + vy * q.d[1] + vz * q.d[2]) / dd;
                    const double tk = a.sigma[q.nu] * xHk * nHk * lk;
                    double ak, outk;
                    attenuate(nin, tk, ak, outk);
                    Rec rc;
                    rc.nout = outk;
                    rc.dx = q.d[0];
                    rc.dy = q.d[1];
                    rc.dz = q.d[2];
                    rc.clk = cv + lk / kCLight;
                    rc.nabs = ak;
                    rc.nin = nin;
                    rc.key = q.key | (static_cast<unsigned long long>(depth) << 8) | (1ull << 7) |
                             static_cast<unsigned long long>(lane);
                    rc.j = static_cast<int>(jk);
                    rc.o = q.nu * a.nrc + r;
                    push_record(a.rec, a.rec_next, a.head, idx1 + w8, rc);
                    const long long tm = jk >> a.lgT;
                    if (!a.list_here) {
                        a.hot[tm] = stamp;
                    } else if (atomicExch(&a.hot[tm], stamp) != stamp) {
                        // the tile's first mark for this forward step: list it
                        const long long at = static_cast<long long>(atomicAdd(
                            reinterpret_cast<unsigned long long*>(&a.cnt[kCntTileList + (a.hop & 1)]), 1ull));
                        const long long j0 = tm * a.T, j1 = (j0 + a.T < a.N) ? j0 + a.T : a.N;
                        a.tlist[at] = make_int4(static_cast<int>(tm), a.rev_off[j0], a.rev_off[j1], 0);
                    }
                }
                break;
            }
            if (depth >= a.max_depth) {
                if (lane == 0) vip_settle(a, q, 1, nrem);
                break;
            }
            q.x[0] = xv[0];
            q.x[1] = xv[1];
            q.x[2] = xv[2];
            q.h = hv;
            q.N = nrem;
            q.c = cv;
        }
    }
}

// --------------------------------------------------------- forward step --

// Working arrays of the forward steps.
// Resting state, updated in place by the workgroup that owns the particle:
//   pk[b]  = {dx, dy, dz, N}, pcl[b] = clock    packet of slot b
//   cm[b]  = cone mask over the neighbours of its particle, written when the
//            packet becomes active
// Moving packets, double-buffered by forward-step parity and read only in the
// forward step after the one that wrote them:
//   mv[b]  = {dx, dy, dz, N / n_c}, mvc[b] = {clock, downstream reception cone}
//   inbox[e], e a receiver-sorted edge i -> j, written by the sender i:
//     tag  = stamp << 1 | 1 if a moving packet of i arrives in a reception
//            cone other than its own index
//     mask = bit (nu*N_RC + p) set: packet (i, nu, p) moves and j is in its cone
// Work marks: hot[tile] = stamp of the forward step in which the tile
// receives packets or records, or has packets leaving.  A stamp numbers the
// forward steps of the whole run, so inboxes and marks are never cleared.
template <typename R>
struct R2 {
    R c, s;
};

template <typename DT>
struct Inbox {
    unsigned int tag;
    DT mask;
};

template <typename R, typename DT>
struct HopArgs {
    long long N;
    int G, nrc, nf, K, rr_bin, rr_on, T, lgT;
    int hop, hop0, max_hops;
    int list0;               // hop 0 runs the tiles of its list (k_mark_hop0), not every tile
    const double* pos;
    const int* rev_off;
    const unsigned int* rev_ik;   // receiver-sorted edges: sender << 6 | position in the sender's list
    const void* rev_v;            // their offsets x_receiver - x_sender (FP32: box units)
    const void* fwd_v;            // offsets x_neighbour - x_particle (FP32: unit vectors); fourth
                                  // component: bits of the edge's receiver-sorted index
    const int* ngb;
    const int* inst_of;
    const double* xHI;
    const double* nH;
    const float* kappa;      // FP32: x_HI n_H L_inst
    const R* floor_b;        // floor in bin units
    const double* h;
    const double* sigma;
    const float* sigmaf;
    R c2;
    double c2d;              // cos^2 of the cone half-angle, FP64 (the exact test)
    float cos_lo, cos_hi;    // FP32: cos(theta) - kConeGuard, cos(theta) + kConeGuard
    R dtc;                   // clock limit in clock units
    const float* clf;        // FP32: L_inst / (c dt) per instance
    const double* U;         // photons per bin unit per instance (1 in FP64)
    const double* scale;     // [n_inst*nf] rescale of in-flight photons at hop 0 (FP32)
    const double* nrr_prev;  // RR photons to emit at hop 0
    const double* rr_pre;    // predecessor RR scheme: arrivals summed per slot of the RR bin (or null)
    const double* wrc;
    const float* wrcf;
    double dt;
    Bin4<R>* pk;
    R* pcl;
    unsigned long long* cm;
    const Bin4<R>* mv_rd;
    const R2<R>* mvc_rd;
    const Inbox<DT>* in_rd;
    const int* hot_rd;
    const int4* tlist;       // this forward step's list of tiles (every tile at hop 0 without
                             // list0): {tile, first and end receiver-sorted edge of its particles, 0}
    int* rest;               // per tile: 1 if a slot held photons after the tile last ran
    long long ntiles;
    int lg_wpb;              // log2 of the wavefronts (tiles) per workgroup: 0, 1 or 2
    unsigned int lds_wave;   // LDS bytes of each wavefront
    Bin4<R>* mv_wr;
    R2<R>* mvc_wr;
    Inbox<DT>* in_wr;
    int* hot_wr;
    double* A;
    double* P;
    double* Fp;              // [N][nf] photons resting in the particle's bins (physical)
    unsigned long long* xr_fx;  // escaped/removed fixed-point accumulators (a full virtual-particle list)
    const double* Ufx;          // their unit per instance
    const Rec* rec;
    const int* rec_next;
    int* head;               // record lists of this forward step, emptied once read
    Vip* vip_out;
    long long vip_cap;
    int list_wr;
    long long* cnt;
    unsigned long long* part;  // [tile][3]: packets moved, bytes, forward steps run (summed per RT step)
    int* listlen;              // [max_hops + 2]: tiles on each forward step's list (the host sizes grids by it)
    int act_rd, act_wr;
};

// Sums of one bin's merge: photons (with a TwoSum compensation term in FP32)
// and the photon-weighted direction and clock.
template <typename R>
struct Acc {
    R n, sx, sy, sz, sc;
    R en;  // compensation of n (FP32 only)
};

template <typename R>
__device__ inline void tsum(R& s, R& e, R x) {
    // Knuth's TwoSum: s + e accumulates x with its rounding error kept in e.
    const R t = s + x;
    const R z = t - s;
    e += (s - (t - z)) + (x - z);
    s = t;
}

// Adds a packet given as its photons n and the products n d and n c.  The
// photon count is TwoSum-compensated in FP32; the weighted direction and clock
// only enter normalised means and are summed plainly.
template <typename R>
__device__ inline void acc_addp(Acc<R>& a, R n, R ndx, R ndy, R ndz, R nc) {
    if constexpr (sizeof(R) == 4)
        tsum(a.n, a.en, n);
    else
        a.n += n;
    a.sx += ndx;
    a.sy += ndy;
    a.sz += ndz;
    a.sc += nc;
}

template <typename R>
__device__ inline void acc_add(Acc<R>& a, R n, R dx, R dy, R dz, R c) {
    acc_addp(a, n, n * dx, n * dy, n * dz, n * c);
}

// FP32 transport: absorbed N_in (1 - e^-tau) and transmitted N_in e^-tau parts
// of a leg without branches.  Below tau = ln 2 the absorbed part is direct,
// from the Taylor series of e^x - 1 to degree 9 (truncation below 2e-8
// relative there); above, the transmitted part is direct, from the hardware
// base-2 exponential.  The other part is the remainder, so they sum to N_in.
__device__ inline void attenuate_f32(float nin, float tau, float& nabs, float& nout) {
    const float x = -tau;
    float p = 1.0f / 362880.0f;
    p = __builtin_fmaf(p, x, 1.0f / 40320.0f);
    p = __builtin_fmaf(p, x, 1.0f / 5040.0f);
    p = __builtin_fmaf(p, x, 1.0f / 720.0f);
    p = __builtin_fmaf(p, x, 1.0f / 120.0f);
    p = __builtin_fmaf(p, x, 1.0f / 24.0f);
    p = __builtin_fmaf(p, x, 1.0f / 6.0f);
    p = __builtin_fmaf(p, x, 0.5f);
    p = __builtin_fmaf(p, x, 1.0f);
    const bool thin = tau < 0.693147182f;
    const float d = thin ? -nin * (p * x) : nin * __builtin_amdgcn_exp2f(x * 1.44269502f);
    const float rest = nin - d;
    nabs = thin ? d : rest;
    nout = thin ? rest : d;
}

template <typename R>
__device__ inline void sum_add(R& s, R& e, R x) {
    if constexpr (sizeof(R) == 4) {
        tsum(s, e, x);
    } else {
        s += x;
    }
}

template <typename R>
__device__ inline R group_sum(R v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
    return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Bit-matrix transpose inside each aligned group of G lanes (G a power of two
// <= 64, the word type wide enough): lane o holds row o (bit c = entry (o, c),
// c < G) and receives column o (bit e = entry (e, o)).  log2(G) rounds, each
// exchanging the off-diagonal halves of 2j x 2j blocks between lanes o and o^j;
// the rounds are written out so that every mask and lane offset is a constant.
// The value of lane (this lane ^ 2^LJ) with the cheapest exchange the
// distance allows: quad permutes for 1 and 2 and a rotation by 8 within a row
// of 16 (DPP, no LDS unit), swizzles for 4 and 16, a permute for 32.
template <int LJ>
__device__ inline unsigned int xor_lane32(unsigned int x) {
    if constexpr (LJ == 0)
        return static_cast<unsigned int>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
    else if constexpr (LJ == 1)
        return static_cast<unsigned int>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
    else if constexpr (LJ == 3)
        return static_cast<unsigned int>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x128, 0xF, 0xF, false));  // row_ror:8
    else if constexpr (LJ == 2)
        return static_cast<unsigned int>(__builtin_amdgcn_ds_swizzle(static_cast<int>(x), 0x101F));  // xor 4 in 32
    else if constexpr (LJ == 4)
        return static_cast<unsigned int>(__builtin_amdgcn_ds_swizzle(static_cast<int>(x), 0x401F));  // xor 16 in 32
    else
        return __shfl_xor(x, 32, 64);
}

template <int LJ, typename W>
__device__ inline W xor_lane(W x) {
    if constexpr (sizeof(W) == 4) {
        return static_cast<W>(xor_lane32<LJ>(static_cast<unsigned int>(x)));
    } else {
        const unsigned int lo = xor_lane32<LJ>(static_cast<unsigned int>(x));
        const unsigned int hi = xor_lane32<LJ>(static_cast<unsigned int>(static_cast<unsigned long long>(x) >> 32));
        return static_cast<W>((static_cast<unsigned long long>(hi) << 32) | lo);
    }
}

// Sum over aligned groups of `width` lanes (a power of two <= 32) in FP32,
// butterfly order from width/2 down to 1 (the order of group_sum above).
template <int LJ>
__device__ inline void group_sum_round(float& v, int width) {
    if ((1 << LJ) < width) v += __uint_as_float(xor_lane32<LJ>(__float_as_uint(v)));
}

__device__ inline float group_sum_f32(float v, int width) {
    group_sum_round<4>(v, width);
    group_sum_round<3>(v, width);
    group_sum_round<2>(v, width);
    group_sum_round<1>(v, width);
    group_sum_round<0>(v, width);
    return v;
}

__device__ inline unsigned long long wave_sum_u64_fast(unsigned long long v) {
    v += xor_lane<5>(v);
    v += xor_lane<4>(v);
    v += xor_lane<3>(v);
    v += xor_lane<2>(v);
    v += xor_lane<1>(v);
    v += xor_lane<0>(v);
    return v;
}

template <int LJ, typename W>
__device__ inline void transpose_round(W& x, int G, int o) {
    constexpr int j = 1 << LJ;
    if constexpr (j < 8 * static_cast<int>(sizeof(W))) {
        if (j < G) {
            constexpr unsigned long long kMask[6] = {0x5555555555555555ull, 0x3333333333333333ull,
                                                     0x0F0F0F0F0F0F0F0Full, 0x00FF00FF00FF00FFull,
                                                     0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
            constexpr W m = static_cast<W>(kMask[LJ]);  // bits c with (c & j) == 0
            const W y = xor_lane<LJ>(x);
            // the lower lane of a pair keeps its bits in m and takes the
            // partner's shifted up; the upper lane keeps ~m and takes them
            // shifted down (selects as bit operations, no branch)
            const W up = static_cast<W>(0) - static_cast<W>((o >> LJ) & 1);
            const W keep = m ^ up;
            const W ys = static_cast<W>(((y >> j) & up) | ((y << j) & ~up));
            x = static_cast<W>((x & keep) | (ys & ~keep));
        }
    }
}

// The same transpose as a loop over the rounds, compact in code and registers:
// the FP64 kernel, whose register budget is tight, runs faster with it.
template <typename W>
__device__ inline W group_transpose_loop(W x, int G, int o) {
    for (int j = G >> 1; j > 0; j >>= 1) {
        W m;  // bits c with (c & j) == 0
        switch (j) {
            case 32: m = static_cast<W>(0x00000000FFFFFFFFull); break;
            case 16: m = static_cast<W>(0x0000FFFF0000FFFFull); break;
            case 8: m = static_cast<W>(0x00FF00FF00FF00FFull); break;
            case 4: m = static_cast<W>(0x0F0F0F0F0F0F0F0Full); break;
            case 2: m = static_cast<W>(0x3333333333333333ull); break;
            default: m = static_cast<W>(0x5555555555555555ull); break;
        }
        const W y = __shfl_xor(x, j, 64);
        x = (o & j) ? static_cast<W>((x & ~m) | ((y & ~m) >> j)) : static_cast<W>((x & m) | ((y & m) << j));
    }
    return x;
}

template <typename W>
__device__ inline W group_transpose(W x, int G, int o) {
    transpose_round<5>(x, G, o);
    transpose_round<4>(x, G, o);
    transpose_round<3>(x, G, o);
    transpose_round<2>(x, G, o);
    transpose_round<1>(x, G, o);
    transpose_round<0>(x, G, o);
    return x;
}

// LDS of a forward-step workgroup (bytes from the start of its dynamic LDS).
// While gathering: a chunk of the tile's incoming edges (their inboxes and
// sender words), the queue of (edge, packet, receiving slot) pairs with
// their contributions, and per particle the two values the attenuation needs.
// Afterwards the same bytes hold, for the particles with active packets, the
// neighbour offsets (receiver-sorted edge index in the fourth component), the
// neighbours and the delivery words.
// Shapes of a forward-step workgroup the autotuner chooses among: incoming
// edges staged per chunk, and (edge, packet) pairs gathered per round in FP32
// (half as many in FP64, at least 64).  Every shape adds a slot's contributions in the same
// order, so they give identical results.
template <int E, int P>
struct HopShape {
    static constexpr int kEdges = E;
    static constexpr int kPairs32 = P;
};
using HopShape0 = HopShape<256, 128>;
using HopShape1 = HopShape<128, 64>;
using HopShape2 = HopShape<512, 256>;
constexpr int kHopShapeKinds = 3;
// Launch configurations the tuner chooses among: shape c % 3, and c / 3 == 1
// packs up to four tiles (independent wavefronts) per workgroup.
constexpr int kHopShapes = 2 * kHopShapeKinds;

template <typename R, typename DT, typename S = HopShape0>
struct HopLds {
    static constexpr int kEdges = S::kEdges;                                       // edges staged at a time
    // pairs gathered at a time (a multiple of the wavefront)
    static constexpr int kPairs = sizeof(R) == 4 ? S::kPairs32 : (S::kPairs32 / 2 > 64 ? S::kPairs32 / 2 : 64);
    static constexpr size_t ik = 0;
    static constexpr size_t tag = ik + 4 * kEdges;    // raw inbox words, loaded straight into LDS
    static constexpr size_t mw = tag + 4 * kEdges;    // [sizeof(DT)/4][kEdges] mask words
    static constexpr size_t dl = mw + sizeof(DT) * kEdges;
    static constexpr size_t eff = dl + sizeof(DT) * kEdges;
    static constexpr size_t nd = eff + sizeof(DT) * kEdges;
    static constexpr size_t desc = (nd + kEdges + 31) / 32 * 32;
    static constexpr size_t val = desc + 4 * kPairs;
    static constexpr size_t part = val + 7 * sizeof(R) * kPairs;
    // Rows of neighbour offsets and neighbours, one per particle.  FP32: 64
    // entries per row (filled by one direct global-to-LDS load per row, lanes
    // past K repeating the last neighbour), offsets padded to 65 against bank
    // conflicts; FP64: K entries, offsets padded to K + 1.
    __host__ __device__ static constexpr int fstride(int K) { return sizeof(R) == 4 ? 65 : K + 1; }
    __host__ __device__ static constexpr int nstride(int K) { return sizeof(R) == 4 ? 64 : K; }
    __host__ __device__ static constexpr size_t ngb_off(int T, int K) {
        return static_cast<size_t>(T) * fstride(K) * 4 * sizeof(R);
    }
    // the rotated reception-cone directions of the step (3 N_RC <= 96 values),
    // after everything else: read by every lane when it bins a packet
    __host__ __device__ static constexpr size_t rcd_off(int T, int K) {
        const size_t g = part + sizeof(R) * (64 + static_cast<size_t>(T));
        const size_t f = ngb_off(T, K) + 4 * static_cast<size_t>(T) * nstride(K);
        return ((g > f ? g : f) + 15) / 16 * 16;
    }
    __host__ __device__ static constexpr size_t bytes(int T, int K) { return rcd_off(T, K) + 96 * sizeof(R); }
};

// One forward step (section 2.1), receiver-sorted.  A workgroup of one
// wavefront owns a tile of T = 64 / G consecutive particles, one lane per slot
// (particle j, bin nu, reception cone r), and runs only if the tile is on this
// forward step's list.  Gathering: the inboxes of the tile's incoming edges
// are staged in LDS; each slot counts the packets that arrive in its cone
// (from LDS alone), a prefix sum lays the (edge, packet, slot) pairs out in
// one queue, and all lanes load and attenuate the queued packets together
// (split equally among the packet's cone members, absorbed 1 - exp(-tau));
// each slot then adds its contributions in edge order.  It merges them with
// the packet that stays and with the records of emission and virtual
// particles (photons add, direction and clock luminosity-weighted); a bin that
// receives nothing keeps its packet as it is.  For a packet that becomes
// active it finds the cone members among j's neighbours and the downstream
// reception cone, writes the delivery masks into the receivers' inboxes and
// marks the tiles that will receive it.  Hop 0 of a step also merges what
// stays (clocks carried over by -dt), the recombination photons of the last
// chemistry step (section 2.2) and the emission records.
template <typename R, typename DT, typename S, bool kExt>
__device__ __forceinline__ void hop_tile(const HopArgs<R, DT>& a, const long long tile, const long long e_t0,
                                         const long long e_t1, const int stamp, const unsigned int tidx,
                                         unsigned char* __restrict__ lds) {
    // e_t0 .. e_t1: the tile's range of receiver-sorted edges
    constexpr bool f32 = sizeof(R) == 4;
    constexpr unsigned long long rsz = sizeof(R);
    using V4 = typename std::conditional<f32, float4, double4>::type;
    using L = HopLds<R, DT, S>;
    constexpr int kP = L::kPairs;

    const int G = a.G, nrc = a.nrc, K = a.K, T = a.T;
    const int lgG = __builtin_ctz(G), lgN = __builtin_ctz(nrc);  // both powers of two
    const long long j0 = tile * T;
    const int jl = tidx >> lgG;
    const int o = tidx & (G - 1);
    const long long j = j0 + jl;
    const bool valid = jl < T && j < a.N;
    const long long s = j * G + o;
    const int nu = o >> lgN;
    const int r = o & (nrc - 1);
    const long long jend = (j0 + T < a.N) ? j0 + T : a.N;
    const int lane = tidx;
    // Gather staging: a chunk of the tile's incoming edges, inbox words and
    // edge words straight from memory into LDS (no registers held, all loads in
    // flight together); lanes past the end load a copy of the last edge.  The
    // first chunk is requested before the tile's own loads, so that both
    // arrive in one round trip.
    unsigned int* e_ik = reinterpret_cast<unsigned int*>(lds + L::ik);
    unsigned int* e_tag = reinterpret_cast<unsigned int*>(lds + L::tag);
    unsigned int* e_mw = reinterpret_cast<unsigned int*>(lds + L::mw);
    auto stage_chunk = [&](long long cb) {
        const long long ne = (e_t1 - cb < L::kEdges) ? e_t1 - cb : L::kEdges;
        const int nrd = static_cast<int>((ne + 63) >> 6);
        for (int i = 0; i < nrd; ++i) {
            const long long t = 64ll * i + lane;
            const long long ts = cb + (t < ne ? t : ne - 1);
            const unsigned int* ws = reinterpret_cast<const unsigned int*>(a.in_rd + ts);
            __builtin_amdgcn_global_load_lds(ws, e_tag + 64 * i, 4, 0, 0);
            for (int w = 0; w < static_cast<int>(sizeof(DT) / 4); ++w)
                __builtin_amdgcn_global_load_lds(ws + offsetof(Inbox<DT>, mask) / 4 + w, e_mw + w * L::kEdges + 64 * i, 4, 0, 0);
            __builtin_amdgcn_global_load_lds(a.rev_ik + ts, e_ik + 64 * i, 4, 0, 0);
        }
    };
    if (!a.hop0 && e_t0 < e_t1) stage_chunk(e_t0);
    // Everything the slot reads of its own particle, and the tile's edge
    // ranges: independent loads, issued together at clamped (always valid)
    // indices before any loaded value is tested.
    const long long jc = valid ? j : j0;
    const long long ia = jc * a.nf + nu;
    const int inst_l = a.inst_of[jc];
    const R flo_l = a.floor_b[jc];
    const int hd_l = a.head[jc];
    const Bin4<R> q0_l = a.pk[jc * G + o];
    const R c0_l = a.pcl[jc * G + o];
    R ka_l, sg_l, nh_l;  // the optical depth's per-particle and per-bin factors
    if constexpr (f32) {
        ka_l = a.kappa[jc];
        sg_l = a.sigmaf[nu];
        nh_l = R(0);
    } else {
        ka_l = a.xHI[jc];
        sg_l = a.sigma[nu];
        nh_l = a.nH[jc];
    }
    const long long my0_l = a.rev_off[jc], my1_l = a.rev_off[jc + 1];
    R* rcd = reinterpret_cast<R*>(lds + L::rcd_off(T, K));
    if (lane < 3 * nrc) rcd[lane] = f32 ? static_cast<R>(a.wrcf[lane]) : static_cast<R>(a.wrc[lane]);
    // per instance: a second, dependent round
    const int inst = valid ? inst_l : 0;
    const double U = f32 ? a.U[inst] : 1.0;
    const float clf_l = f32 ? a.clf[inst] : 0.0f;
    // algorithmic bytes this lane moves (slot state, gathered packets, edges)
    unsigned long long nbytes = 0;

    Acc<R> acc = {};
    int narr = 0;            // packets merged into the bin besides the one that stays
    R asum = 0, aerr = 0, psum = 0, perr = 0;
    R rsum = 0;  // photons of arrivals removed by the barrier on their way
    Bin4<R> q0 = {};
    R c0 = 0;
    bool have_stay = false, departed = false;
    const R flo = valid ? flo_l : R(0);
    const int hd = valid ? hd_l : -1;
    q0.x = valid ? q0_l.x : R(0);  // selects, so that the loads stay up front
    q0.y = valid ? q0_l.y : R(0);
    q0.z = valid ? q0_l.z : R(0);
    q0.n = valid ? q0_l.n : R(0);
    c0 = valid ? c0_l : R(0);
    if (valid) {
        nbytes += 5 * rsz;
        if (q0.n > R(0)) {
            if (a.hop0) {
                if constexpr (f32) q0.n = static_cast<R>(static_cast<double>(q0.n) * a.scale[inst * a.nf + nu]);
                c0 = c0 - a.dtc;
                have_stay = q0.n > R(0);
            } else if (!(c0 < a.dtc)) {
                have_stay = true;
            } else {
                departed = true;  // it moved on in this forward step
            }
        }
        if (have_stay) acc_add(acc, q0.n, q0.x, q0.y, q0.z, c0);
        if (a.hop0 && a.rr_on && nu == a.rr_bin) {
            const double nr = a.nrr_prev[j];
            if (nr > 0.0) {
                const R per = static_cast<R>(nr / static_cast<double>(nrc) / U);
                if constexpr (f32)
                    acc_add(acc, per, a.wrcf[3 * r], a.wrcf[3 * r + 1], a.wrcf[3 * r + 2], R(0));
                else
                    acc_add(acc, per, R(a.wrc[3 * r]), R(a.wrc[3 * r + 1]), R(a.wrc[3 * r + 2]), R(0));
                ++narr;
            }
        }
        if constexpr (kExt) {
            if (a.hop0 && a.rr_pre && nu == a.rr_bin) {
                // the predecessor RR scheme's arrivals in this cone, summed in edge order
                const double* pr = a.rr_pre + 6 * (j * nrc + r);
                if (pr[5] > 0.0) {
                    if constexpr (f32) {
                        const double iu = 1.0 / U;
                        acc_addp(acc, static_cast<R>(pr[0] * iu), static_cast<R>(pr[1] * iu), static_cast<R>(pr[2] * iu),
                                 static_cast<R>(pr[3] * iu), static_cast<R>(pr[4] * iu / a.dt));
                    } else {
                        acc_addp(acc, R(pr[0]), R(pr[1]), R(pr[2]), R(pr[3]), R(pr[4]));
                    }
                    ++narr;
                }
            }
        }
    }
    if (!a.hop0) {
        DT* e_dl = reinterpret_cast<DT*>(lds + L::dl);
        DT* e_ef = reinterpret_cast<DT*>(lds + L::eff);
        unsigned char* e_nd = lds + L::nd;
        unsigned int* pdesc = reinterpret_cast<unsigned int*>(lds + L::desc);
        R* pval = reinterpret_cast<R*>(lds + L::val);  // [7][kP]
        // per (particle, bin): FP32 sigma_nu kappa, FP64 sigma_nu x_HI (the
        // first product of the optical depth); per particle: FP32 L/(c dt), FP64 n_H
        R* pa = reinterpret_cast<R*>(lds + L::part);
        R* pb = pa + 64;
        if (valid && r == 0) {
            pa[jl * a.nf + nu] = sg_l * ka_l;
            if (o == 0) pb[jl] = f32 ? static_cast<R>(clf_l) : nh_l;
        }
        const long long my0 = valid ? my0_l : 0, my1 = valid ? my1_l : 0;
        const unsigned int prev = static_cast<unsigned int>(stamp - 1);
        const DT gm = static_cast<DT>(nrc >= 8 * static_cast<int>(sizeof(DT)) ? ~DT(0) : ((DT(1) << nrc) - DT(1)));
        const int gbase_s = lane & ~(G - 1);
        const unsigned long long gmask_s = G >= 64 ? ~0ull : ((1ull << G) - 1ull);
        for (long long cb = e_t0; cb < e_t1; cb += L::kEdges) {
            const long long ne = (e_t1 - cb < L::kEdges) ? e_t1 - cb : L::kEdges;
            bool snd = false;
            if (cb != e_t0) stage_chunk(cb);  // the first chunk is already on its way
            __builtin_amdgcn_s_waitcnt(0);
            wave_sync();
            for (long long t = lane; t < ne; t += 64) {
                const unsigned int wtag = e_tag[t];
                DT wmask = static_cast<DT>(e_mw[t]);
                if constexpr (sizeof(DT) == 8) wmask |= static_cast<DT>(e_mw[L::kEdges + t]) << 32;
                const DT m = (wtag >> 1) == prev ? wmask : DT(0);
                const bool nd = (wtag & 1u) != 0;
                // effective mask: bit (nu, r) set if the edge may bring a packet
                // into reception cone r; a sender with packets arriving off
                // their own index may reach any cone of a bin it delivers in
                DT ef = m;
                if (nd && m != DT(0)) {
                    ef = DT(0);
                    for (int f = 0; f < a.nf; ++f)
                        if ((m >> (f * nrc)) & gm) ef |= gm << (f * nrc);
                    snd = true;
                }
                e_dl[t] = m;
                e_ef[t] = ef;
                e_nd[t] = static_cast<unsigned char>(nd);
                nbytes += sizeof(Inbox<DT>) + 4;
            }
            wave_sync();
            const bool any_nd = __ballot(snd) != 0;
            const long long lo = my0 > cb ? my0 : cb;
            const long long hi = my1 < cb + ne ? my1 : cb + ne;
            // hit mask of this slot over a segment of up to 64 of its particle's
            // edges: the particle's lanes read its edges G at a time (lane o:
            // edge o's effective mask, a row) and a bit-matrix transpose hands
            // each slot lane its bit of every edge (a column).  A particle's
            // lanes share lo and hi, so they run the same rounds.
            const int nseg = hi > lo ? static_cast<int>((hi - lo + 63) >> 6) : 0;
            auto seg_hit = [&](int sg) {
                const long long sb = lo + 64ll * sg;
                const int len = static_cast<int>(hi - sb < 64 ? hi - sb : 64);
                unsigned long long h = 0;
                for (int k = 0; k * G < 64; ++k) {
                    const int idx = k * G + o;
                    DT v = idx < len ? static_cast<DT>(e_ef[sb - cb + idx] & static_cast<DT>(gmask_s)) : DT(0);
                    v = f32 ? group_transpose(v, G, o) : group_transpose_loop(v, G, o);
                    h |= (static_cast<unsigned long long>(v) & gmask_s) << (k * G);
                }
                return h;
            };
            const unsigned long long h0 = nseg > 0 ? seg_hit(0) : 0ull;  // usually the only segment
            // this slot's arriving (edge, packet) pairs, in edge order
            auto each_pair = [&](auto&& f) {
                for (int sg = 0; sg < nseg; ++sg) {
                    unsigned long long h = sg == 0 ? h0 : seg_hit(sg);
                    while (h) {
                        const int u = __builtin_ctzll(h);
                        h &= h - 1ull;
                        const int t = static_cast<int>(lo + 64ll * sg - cb) + u;
                        if (!e_nd[t]) {
                            f(t, r);
                            continue;
                        }
                        DT m = (e_dl[t] >> (nu * nrc)) & gm;
                        while (m != DT(0)) {
                            const int pp = static_cast<int>(__builtin_ctzll(static_cast<unsigned long long>(m)));
                            m &= m - DT(1);
                            f(t, pp);
                        }
                    }
                }
            };
            int np = 0;
            if (any_nd) {
                each_pair([&](int, int) { ++np; });
            } else {
                for (int sg = 0; sg < nseg; ++sg) np += __popcll(sg == 0 ? h0 : seg_hit(sg));
            }
            // exclusive prefix sum over the wavefront
            int incl = np;
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const int M = __shfl(incl, 63, 64);
            const int off0 = incl - np;
            for (int base = 0; base < M; base += kP) {
                if (!any_nd) {
                    // no sender arrives off its own cone index: each hit edge
                    // brings exactly the slot's own packet index, no LDS lookup
                    int q = off0;
                    for (int sg = 0; sg < nseg; ++sg) {
                        unsigned long long h = sg == 0 ? h0 : seg_hit(sg);
                        const unsigned int tb = static_cast<unsigned int>(lo + 64ll * sg - cb);
                        while (h) {
                            const unsigned int u = static_cast<unsigned int>(__builtin_ctzll(h));
                            h &= h - 1ull;
                            if (q >= base && q < base + kP)
                                pdesc[q - base] = ((tb + u) << 14) | (static_cast<unsigned int>(r) << 8) | tidx;
                            ++q;
                        }
                    }
                } else {
                    // every lane takes part: the transpose needs all of a particle's lanes
                    int q = off0;
                    each_pair([&](int t, int pp) {
                        if (q >= base && q < base + kP)
                            pdesc[q - base] = (static_cast<unsigned int>(t) << 14) | (static_cast<unsigned int>(pp) << 8) | tidx;
                        ++q;
                    });
                }
                wave_sync();
                const int nr = (M - base < kP) ? M - base : kP;
                // load and attenuate the queued packets (all lanes; loads first)
                constexpr int kPer = kP / 64;
                Bin4<R> q[kPer];
                R2<R> qc[kPer];
                V4 v[kPer];
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int u = lane + 64 * i;
                    if (u < nr) {
                        const unsigned int d = pdesc[u];
                        const int t = static_cast<int>(d >> 14), pp = static_cast<int>(d >> 8) & 63, sl = static_cast<int>(d & 255u);
                        const int so = sl & (G - 1);
                        const long long tt = (static_cast<long long>(e_ik[t] >> 6) << lgG) + (so & ~(nrc - 1)) + pp;
                        qc[i] = a.mvc_rd[tt];
                        q[i] = a.mv_rd[tt];
                        v[i] = static_cast<const V4*>(a.rev_v)[cb + t];
                    }
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int u = lane + 64 * i;
                    if (u < nr) {
                        const unsigned int d = pdesc[u];
                        const int t = static_cast<int>(d >> 14), sl = static_cast<int>(d & 255u);
                        const int sjl = sl >> lgG, so = sl & (G - 1), snu = so >> lgN, sr = so & (nrc - 1);
                        nbytes += 10 * rsz;
                        if (e_nd[t] && static_cast<int>(qc[i].s) != sr) {
                            pval[6 * kP + u] = R(-1);  // arrives in another cone of the particle
                            continue;
                        }
                        R tau, cl, nabs, nout;
                        if constexpr (f32) {
                            // path length: the offset along the packet's (unit) direction
                            const float aa = __builtin_fmaf(v[i].z, q[i].z, __builtin_fmaf(v[i].y, q[i].y, v[i].x * q[i].x));
                            const float qq = __builtin_fmaf(q[i].z, q[i].z, __builtin_fmaf(q[i].y, q[i].y, q[i].x * q[i].x));
                            const float l = aa * __builtin_amdgcn_rsqf(qq);
                            tau = pa[sjl * a.nf + snu] * l;
                            cl = __builtin_fmaf(l, pb[sjl], qc[i].c);
                            attenuate_f32(q[i].n, tau, nabs, nout);
                        } else {
                            const R aa = static_cast<R>(v[i].x) * q[i].x + static_cast<R>(v[i].y) * q[i].y +
                                         static_cast<R>(v[i].z) * q[i].z;
                            const R l = aa / sqrt(q[i].x * q[i].x + q[i].y * q[i].y + q[i].z * q[i].z);
                            tau = pa[sjl * a.nf + snu] * pb[sjl] * l;
                            cl = qc[i].c + l / kCLight;
                            attenuate(q[i].n, tau, nabs, nout);
                        }
                        // FP32: the merge's products, formed here on all lanes at once
                        pval[u] = nout;
                        pval[kP + u] = f32 ? nout * q[i].x : q[i].x;
                        pval[2 * kP + u] = f32 ? nout * q[i].y : q[i].y;
                        pval[3 * kP + u] = f32 ? nout * q[i].z : q[i].z;
                        pval[4 * kP + u] = f32 ? nout * cl : cl;
                        // an edge that meets the barrier removes the packet on the
                        // way (marked by nin = -2, its photons where nabs would be)
                        const bool cut = kExt && v[i].w != static_cast<decltype(v[i].w)>(0);
                        pval[5 * kP + u] = cut ? q[i].n : nabs;
                        pval[6 * kP + u] = cut ? R(-2) : q[i].n;
                    }
                }
                wave_sync();
                // this slot's contributions, in order
                const int qa = off0 > base ? off0 : base;
                const int qb = (off0 + np < base + nr) ? off0 + np : base + nr;
                for (int qq = qa; qq < qb; ++qq) {
                    const int u = qq - base;
                    if constexpr (f32) {
                        // all seven values read at once; a packet that arrives in
                        // another cone of the particle (marked by nin < 0) adds
                        // exact zeros, which leave the sums bit for bit unchanged
                        const R nin = pval[6 * kP + u];
                        const R v0 = pval[u], v1 = pval[kP + u], v2 = pval[2 * kP + u], v3 = pval[3 * kP + u],
                                v4 = pval[4 * kP + u], v5 = pval[5 * kP + u];
                        const bool ok = nin >= R(0);
                        if constexpr (kExt) rsum += nin == R(-2) ? v5 : R(0);
                        sum_add(asum, aerr, ok ? v5 : R(0));
                        sum_add(psum, perr, ok ? nin : R(0));
                        acc_addp(acc, ok ? v0 : R(0), ok ? v1 : R(0), ok ? v2 : R(0), ok ? v3 : R(0), ok ? v4 : R(0));
                        narr += ok ? 1 : 0;
                    } else {
                        const R nin = pval[6 * kP + u];
                        if (nin < R(0)) {
                            if (kExt && nin == R(-2)) rsum += pval[5 * kP + u];
                            continue;
                        }
                        sum_add(asum, aerr, pval[5 * kP + u]);
                        sum_add(psum, perr, nin);
                        acc_add(acc, pval[u], pval[kP + u], pval[2 * kP + u], pval[3 * kP + u], pval[4 * kP + u]);
                        ++narr;
                    }
                }
                wave_sync();  // the LDS is reused
            }
        }
    }
    if (valid) {
        // records of emission and virtual particles, in key order
        if (hd >= 0) {
            unsigned long long last = 0;
            bool first = true;
            for (;;) {
                unsigned long long best = ~0ull;
                int bidx = -1;
                for (int qi = hd; qi >= 0; qi = a.rec_next[qi]) {
                    const int ro = a.rec[qi].o;
                    const bool mine = (ro == o) || (ro < 0 && (-1 - ro) == nu && r == 0);
                    if (!mine) continue;
                    const unsigned long long k = a.rec[qi].key;
                    if ((first || k > last) && k < best) {
                        best = k;
                        bidx = qi;
                    }
                }
                if (bidx < 0) break;
                const Rec rc = a.rec[bidx];
                nbytes += sizeof(Rec);
                last = best;
                first = false;
                sum_add(asum, aerr, static_cast<R>(rc.nabs / U));
                if (rc.o >= 0) {
                    sum_add(psum, perr, static_cast<R>(rc.nin / U));
                    acc_add(acc, static_cast<R>(rc.nout / U), static_cast<R>(rc.dx), static_cast<R>(rc.dy),
                            static_cast<R>(rc.dz), static_cast<R>(f32 ? rc.clk / a.dt : rc.clk));
                    ++narr;
                }
            }
        }
    }
    // the bin's packet: merged if anything arrived, otherwise the one that stays
    R nn = 0, dx = 0, dy = 0, dz = 0, cn = 0;
    if (narr == 0) {
        if (have_stay) {
            nn = q0.n;
            dx = q0.x;
            dy = q0.y;
            dz = q0.z;
            cn = c0;
        }
    } else {
        const R an = acc.n + acc.en, sx = acc.sx, sy = acc.sy, sz = acc.sz, sc = acc.sc;
        if (an > R(0)) {
            nn = an;
            const R s2 = sx * sx + sy * sy + sz * sz;
            if (f32 && s2 > R(1e-30)) {
                const R inv = __builtin_amdgcn_rsqf(static_cast<float>(s2));
                dx = sx * inv;
                dy = sy * inv;
                dz = sz * inv;
            } else if (s2 > R(0)) {
                const R nr = sqrt(s2);
                dx = sx / nr;
                dy = sy / nr;
                dz = sz / nr;
            } else {
                if constexpr (f32) {
                    dx = a.wrcf[3 * r];
                    dy = a.wrcf[3 * r + 1];
                    dz = a.wrcf[3 * r + 2];
                } else {
                    dx = a.wrc[3 * r];
                    dy = a.wrc[3 * r + 1];
                    dz = a.wrc[3 * r + 2];
                }
            }
            cn = (f32 && an > R(1e-30)) ? sc * static_cast<R>(__builtin_amdgcn_rcpf(static_cast<float>(an))) : sc / an;
        }
    }
    bool floored = false;
    if (valid && nn > R(0) && nn < flo) {
        sum_add(asum, aerr, nn);
        nn = 0;
        dx = dy = dz = cn = 0;
        floored = true;
    }
    // absorbed / passing photons of (j, nu): sum over the n_rc lanes
    R ag, pg;
    if constexpr (f32) {
        ag = group_sum_f32(asum + aerr, nrc);
        pg = group_sum_f32(psum + perr, nrc);
    } else {
        ag = group_sum(asum + aerr, nrc);
        pg = group_sum(psum + perr, nrc);
    }
    // added in place (one lane per (j, nu) and launch, so the sum is the
    // plain A + ag U): no register holds the old values through the tile
    if (valid && r == 0 && (ag != R(0) || pg != R(0))) {
        unsafeAtomicAdd(&a.A[ia], static_cast<double>(ag) * U);
        unsafeAtomicAdd(&a.P[ia], static_cast<double>(pg) * U);
        nbytes += 32;
    }
    // arrivals the barrier removed: one set of atomics per (instance, bin),
    // in the (rare) wavefronts that saw any
    if constexpr (kExt) {
        if (__ballot(valid && rsum > R(0)) != 0ull)
            fx_add3_wave(a.xr_fx, (static_cast<long long>(inst) * a.nf + nu) * 2 + 1,
                         valid ? static_cast<double>(rsum) * U / a.Ufx[inst] : 0.0, valid && rsum > R(0), a.cnt);
    }
    // photons resting in (j, nu) after this forward step, for the ledger's
    // in-flight total (a tile's bins change only when it runs)
    const double fg = group_sum(valid ? static_cast<double>(nn) * U : 0.0, nrc);
    if (valid && r == 0) {
        a.Fp[ia] = fg;
        nbytes += 8;
    }
    // next forward step: cone members and downstream reception cone.  The
    // lanes of a particle with an active packet stage its neighbour offsets
    // (with the receiver-sorted index of each edge) and its neighbours.
    const bool act = valid && nn > R(0) && cn < a.dtc;
    wave_sync();  // the gather's LDS is free again
    const bool tile_act = __ballot(act) != 0;
    if (valid && o == 0 && hd >= 0) a.head[j] = -1;  // every lane of j has read its records
    if (tile_act && tidx == 0) a.hot_wr[tile] = stamp + 1;  // its leaving packets empty their bins
    const int gbase = lane & ~(G - 1);
    const unsigned long long gmaskG = G >= 64 ? ~0ull : ((1ull << G) - 1ull);
    const unsigned long long wact = __ballot(act);
    const bool pact = ((wact >> gbase) & gmaskG) != 0;
    V4* fj = reinterpret_cast<V4*>(lds) + static_cast<long long>(jl) * L::fstride(K);
    int* nj = reinterpret_cast<int*>(lds + L::ngb_off(T, K)) + static_cast<long long>(jl) * L::nstride(K);
    if constexpr (f32) {
        // direct global-to-LDS loads (4 bytes per lane, all lanes, the row
        // choice uniform) of the rows of particles with an active packet:
        // the 4K words of the offsets, then the K neighbours; lanes past the
        // end repeat the last word, which the row padding absorbs
        const int nwd = 4 * K;
        for (int rw = 0; rw < T; ++rw) {
            if (((wact >> (rw * G)) & gmaskG) == 0) continue;
            const long long jr = j0 + rw;
            const unsigned int* fsrc = reinterpret_cast<const unsigned int*>(static_cast<const float4*>(a.fwd_v) + jr * K);
            unsigned int* fdst = reinterpret_cast<unsigned int*>(reinterpret_cast<V4*>(lds) + rw * L::fstride(K));
            for (int w0 = 0; w0 < nwd; w0 += 64) {
                const int w = w0 + lane < nwd ? w0 + lane : nwd - 1;
                __builtin_amdgcn_global_load_lds(fsrc + w, fdst + w0, 4, 0, 0);
            }
            const int kk = lane < K ? lane : K - 1;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const unsigned int*>(a.ngb + jr * K + kk),
                                             reinterpret_cast<unsigned int*>(lds + L::ngb_off(T, K)) + rw * L::nstride(K), 4, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
        if (pact && o == 0) nbytes += static_cast<unsigned long long>(K) * (4 * rsz + 4);
    } else if (pact) {
        const V4* src = static_cast<const V4*>(a.fwd_v) + j * K;
        const int* sn = a.ngb + j * K;
        // kStage neighbours per lane in flight at once, then into LDS
        constexpr int kStage = 4;
        for (int kb = o; kb < K; kb += kStage * G) {
            V4 f[kStage];
            int nb[kStage];
#pragma unroll
            for (int u = 0; u < kStage; ++u) {
                const int k = min(kb + u * G, K - 1);  // loads in one block, no branch
                f[u] = src[k];
                nb[u] = sn[k];
            }
#pragma unroll
            for (int u = 0; u < kStage; ++u) {
                const int k = kb + u * G;
                if (k < K) {
                    fj[k] = f[u];
                    nj[k] = nb[u];
                }
            }
        }
        if (o == 0) nbytes += static_cast<unsigned long long>(K) * (4 * rsz + 4);
    }
    wave_sync();  // a particle's lanes lie in one wavefront
    unsigned long long cmw = 0;
    int tgt = r;
    if (act) {
        if constexpr (f32) {
            // bit k: neighbour k is a cone member; the bits enter from the
            // highest neighbour down (m = 2m + bit), in two 32-bit halves.
            // The FP32 cosine (unit vectors rounded once, fused products)
            // is within kConeGuard / 4 of the exact one, so it decides every
            // test outside the band cos(theta) -+ kConeGuard; the few inside
            // it are decided by the FP64 test on the FP64 positions, the
            // test of the FP64 transport, so both precisions take the same
            // decision for the same direction.
            unsigned int mh = 0, ml = 0, nh = 0, nl = 0;
            int k = K - 1;
            for (; k >= 32; --k) {
                const V4 w = fj[k];
                const float cv = __builtin_fmaf(w.z, dz, __builtin_fmaf(w.y, dy, w.x * dx));
                mh = mh + mh + (cv >= a.cos_hi ? 1u : 0u);
                nh = nh + nh + (cv >= a.cos_lo ? 1u : 0u);
            }
#pragma unroll 8
            for (; k >= 0; --k) {
                const V4 w = fj[k];
                const float cv = __builtin_fmaf(w.z, dz, __builtin_fmaf(w.y, dy, w.x * dx));
                ml = ml + ml + (cv >= a.cos_hi ? 1u : 0u);
                nl = nl + nl + (cv >= a.cos_lo ? 1u : 0u);
            }
            cmw = (static_cast<unsigned long long>(mh) << 32) | ml;
            unsigned long long band = ((static_cast<unsigned long long>(nh) << 32) | nl) ^ cmw;
            if (band) {
                const double ddx = dx, ddy = dy, ddz = dz;
                const double px = a.pos[3 * j], py = a.pos[3 * j + 1], pz = a.pos[3 * j + 2];
                while (band) {
                    const int kb = __builtin_ctzll(band);
                    band &= band - 1ull;
                    const long long nb = nj[kb];
                    if (in_cone(a.pos[3 * nb] - px, a.pos[3 * nb + 1] - py, a.pos[3 * nb + 2] - pz, ddx, ddy, ddz, a.c2d))
                        cmw |= 1ull << kb;
                }
            }
            // reception cone: the FP32 argmax unless the two largest dot
            // products lie within kConeGuard, then the FP64 argmax
            tgt = nearest_direction_guarded(static_cast<const R*>(rcd), a.wrc, nrc, dx, dy, dz);
        } else {
#pragma unroll 8
            for (int k = 0; k < K; ++k) {
                const V4 w = fj[k];
                if (in_cone(w.x, w.y, w.z, dx, dy, dz, a.c2)) cmw |= 1ull << k;
            }
            tgt = nearest_direction(static_cast<const R*>(rcd), nrc, dx, dy, dz);
        }
    }
    const bool send = act && cmw != 0;
    const bool vip = act && cmw == 0;
    const int nc = __popcll(cmw);
    // delivery words: for each neighbour k, the packets of the particle that
    // reach it; written into the receivers' inboxes, whose tiles are marked
    // for the next forward step
    const unsigned long long wsend = __ballot(send);
    const bool psend = ((wsend >> gbase) & gmaskG) != 0;
    const bool offdiag = __ballot(send && tgt != r) & (gmaskG << gbase);
    if (wsend) {
        // row o: the sending slot o's cone bits for neighbours k0..k0+G-1;
        // transposed, lane o holds the delivery word of neighbour k0 + o
        const unsigned long long cs = send ? cmw : 0ull;
        Inbox<DT> ib;
        ib.tag = (static_cast<unsigned int>(stamp) << 1) | (offdiag ? 1u : 0u);
        for (int k0 = 0; k0 < K; k0 += G) {
            const DT w0 = static_cast<DT>((cs >> k0) & gmaskG);
            const DT w = f32 ? group_transpose(w0, G, o) : group_transpose_loop(w0, G, o);
            const int k = k0 + o;
            if (psend && k < K && w != DT(0)) {
                ib.mask = w;
                long long e;
                if constexpr (f32)
                    e = __float_as_int(fj[k].w);
                else
                    e = __double_as_longlong(fj[k].w);
                a.in_wr[e] = ib;
                a.hot_wr[nj[k] >> a.lgT] = stamp + 1;
                nbytes += sizeof(Inbox<DT>) + 4;
            }
        }
    }
    // virtual particles of this wavefront's empty cones: one list atomic per wavefront
    const unsigned long long wvip = __ballot(vip);
    long long vbase = 0;
    if (wvip) {
        const int ld = __ffsll(static_cast<long long>(wvip)) - 1;
        if (lane == ld)
            vbase = static_cast<long long>(atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntVipCnt0 + a.list_wr]),
                                                     static_cast<unsigned long long>(__popcll(wvip))));
        vbase = __shfl(vbase, ld, 64);
    }
    if (valid) {
        if (a.hop0 || narr > 0 || departed || floored) {
            Bin4<R> w;
            w.x = dx;
            w.y = dy;
            w.z = dz;
            w.n = nn;
            a.pk[s] = w;
            a.pcl[s] = cn;
            nbytes += 5 * rsz;
        }
        if (act) {
            a.cm[s] = cmw;
            nbytes += 8;
        }
        if (send) {
            Bin4<R> w;
            w.x = dx;
            w.y = dy;
            w.z = dz;
            w.n = nn / static_cast<R>(nc);
            a.mv_wr[s] = w;
            R2<R> wc;
            wc.c = cn;
            wc.s = static_cast<R>(tgt);
            a.mvc_wr[s] = wc;
            nbytes += 6 * rsz;
        }
        if (vip) {
            const long long v = vbase + __popcll(wvip & ((1ull << lane) - 1ull));
            if (v >= a.vip_cap) {
                // no room to follow it: its photons leave the transport as removed
                atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagVipOverflow));
                fx_add3(a.xr_fx + 3 * ((static_cast<long long>(inst) * a.nf + nu) * 2 + 1), static_cast<double>(nn) * U / a.Ufx[inst],
                        a.cnt);
            } else {
                Vip q;
                q.x[0] = a.pos[3 * j];
                q.x[1] = a.pos[3 * j + 1];
                q.x[2] = a.pos[3 * j + 2];
                q.h = a.h[j];
                q.d[0] = dx;
                q.d[1] = dy;
                q.d[2] = dz;
                q.N = static_cast<double>(nn) * U;
                q.c = f32 ? static_cast<double>(cn) * a.dt : static_cast<double>(cn);
                q.nu = nu;
                q.inst = inst;
                q.ec = -1;
                q.ek = 0;
                q.tag = kTagVipT;
                q.ida = static_cast<unsigned int>(j);
                q.idb = ((static_cast<unsigned int>(a.hop + 1) & 0xFFFu) << 20) | ((static_cast<unsigned int>(o) & 0xFFFFu) << 4);
                q.xr = s;
                q.xr_emis = 0;
                q.key = (1ull << 62) | (static_cast<unsigned long long>(s) << 12);
                a.vip_out[v] = q;
            }
        }
    }
    // whether a packet moves next step (a flag, no count: plain stores), and
    // the tile's running tallies of packets moved, bytes and steps run
    if (tile_act && lane == 0) a.cnt[kCntAct0 + kCntLine * a.act_wr] = 1;
    // whether photons stay in this tile's bins: the next RT step's first
    // forward step runs it then (it also runs the tiles with records or RR)
    const bool resting = __ballot(valid && nn > R(0)) != 0ull;
    if (lane == 0) a.rest[tile] = resting ? 1 : 0;
    const unsigned long long nupd = __popcll(__ballot(departed));
    const unsigned long long wb = f32 ? wave_sum_u64_fast(nbytes) : wave_sum_u64(nbytes);
    // the tile's running tallies, added in place (the tile's own entries)
    if (lane < 3) atomicAdd(&a.part[3 * tile + lane], lane == 0 ? nupd : (lane == 1 ? wb : 1ull));
    // every LDS read of this tile has been consumed before the next tile stages
    __builtin_amdgcn_s_waitcnt(0);
    wave_sync();
}

// The forward-step kernel: workgroups of a.wpb independent wavefronts, one
// tile each, each wavefront with its own share of the LDS.  A forward step
// runs the tiles of its list (hop 0 with the predecessor RR scheme: every
// tile), packed into the first workgroups of the launch, so the real work is
// dispatched first and the surplus workgroups read one counter and exit.
// Workgroups are dispatched round-robin over the 8 XCDs; xcd_block gives each
// XCD a contiguous share of the list (sorted within each chunk of marks), so
// that neighbouring particles share that XCD's L2.  The
// launch-level flags are read once: a launch past the last forward step of an
// RT step, or past the cap, runs no tile.
// kExt: the variant for the rarely used features, a barrier disk (its edges
// carry a flag, see k_barrier_edges) and the predecessor RR scheme's arrivals
// at the first forward step; the plain variant reads neither
template <typename R, typename DT, typename S, bool kExt>
__global__ __launch_bounds__(256) void k_hop(HopArgs<R, DT> a) {
    extern __shared__ __align__(32) unsigned char lds_all[];
    const long long c_done = a.cnt[kCntDone];
    const long long c_act = a.cnt[kCntAct0 + kCntLine * a.act_rd];
    const long long c_serial = a.cnt[kCntSerial];
    const long long c_list = a.cnt[kCntTileList + (a.hop & 1)];
    const int stamp = static_cast<int>(c_serial) + a.hop;  // of this forward step
    // a step halted on the device (steps replayed from graphs) also sets the
    // done flag, which its hop 0 otherwise never sees: the launch is idle
    const bool idle = (c_done != 0) | ((a.hop0 == 0) & (c_act == 0));
    const bool capped = (a.hop0 == 0) & !idle & (a.hop > a.max_hops);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (idle) {
            a.cnt[kCntDone] = 1;
        } else if (capped) {
            atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagHopCap));
        } else {
            if (!a.hop0) {
                a.cnt[kCntHops] += 1;
                a.cnt[kCntHopsStep] += 1;
            }
            a.cnt[kCntRec] = 0;   // records of this step were all linked before launch
            a.cnt[kCntDeep] = 0;  // and its virtual particles all handled
            // the next forward step's list count starts from zero
            a.cnt[kCntTileList + ((a.hop + 1) & 1)] = 0;
            if (!a.hop0 || a.list0) a.listlen[a.hop] = static_cast<int>(c_list);
        }
    }
    // 32-bit arithmetic and shifts only: every workgroup, also the surplus
    // ones, runs this before it exits.  The grid may be smaller than the list
    // (sized from earlier steps): k_hop_tail takes the tiles past its end.
    const bool every = a.hop0 && !a.list0;  // hop 0 without a list runs every tile
    const unsigned int n = static_cast<unsigned int>(every ? a.ntiles : (c_list < a.ntiles ? c_list : a.ntiles));
    const unsigned int nb0 = (n + (1u << a.lg_wpb) - 1u) >> a.lg_wpb;  // workgroups' worth of tiles
    const unsigned int nb = nb0 < gridDim.x ? nb0 : gridDim.x;          // of them in this grid
    if (idle | capped | (blockIdx.x >= nb)) return;
    const unsigned int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
    const unsigned int e = (xcd_block32(blockIdx.x, nb) << a.lg_wpb) + wv;
    if (e >= n) return;
    long long tile, e_t0, e_t1;
    if (every) {
        tile = e;
        const long long tj0 = tile * a.T;
        const long long tj1 = (tj0 + a.T < a.N) ? tj0 + a.T : a.N;
        e_t0 = a.rev_off[tj0];
        e_t1 = a.rev_off[tj1];
    } else {
        const int4 w = a.tlist[e];  // the tile and its edge range in one load
        tile = w.x;
        e_t0 = static_cast<unsigned int>(w.y);
        e_t1 = static_cast<unsigned int>(w.z);
    }
    hop_tile<R, DT, S, kExt>(a, tile, e_t0, e_t1, stamp, threadIdx.x & 63u, lds_all + static_cast<size_t>(wv) * a.lds_wave);
}

// The tiles of a forward step's list past the end of k_hop's grid (a grid sized
// from earlier steps' lists, so that launches dispatch few workgroups that
// have nothing to do): a small grid takes them in turn.  Usually there are
// none and every workgroup exits at once.  No step bookkeeping here.
template <typename R, typename DT, typename S, bool kExt>
__global__ __launch_bounds__(256) void k_hop_tail(HopArgs<R, DT> a, unsigned int covered) {
    extern __shared__ __align__(32) unsigned char lds_all[];
    const long long c_done = a.cnt[kCntDone];
    const long long c_act = a.cnt[kCntAct0 + kCntLine * a.act_rd];
    const long long c_serial = a.cnt[kCntSerial];
    const long long c_list = a.cnt[kCntTileList + (a.hop & 1)];
    const int stamp = static_cast<int>(c_serial) + a.hop;
    const bool idle = (c_done != 0) | ((a.hop0 == 0) & (c_act == 0));
    const unsigned int n = static_cast<unsigned int>(c_list < a.ntiles ? c_list : a.ntiles);
    if (idle | (a.hop > a.max_hops) | (n <= covered)) return;
    const unsigned int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (unsigned int g = (covered >> a.lg_wpb) + blockIdx.x;; g += gridDim.x) {
        const unsigned int e = (g << a.lg_wpb) + wv;
        if (e >= n) break;
        const int4 w = a.tlist[e];
        hop_tile<R, DT, S, kExt>(a, w.x, static_cast<unsigned int>(w.y), static_cast<unsigned int>(w.z), stamp,
                                 threadIdx.x & 63u, lds_all + static_cast<size_t>(wv) * a.lds_wave);
    }
}


// The marks of an RT step's first forward step (act_rd < 0 in k_tile_list then
// lists them): a tile runs if photons rest in its bins (flag left by its last
// run), or one of its particles has records to consume (emission, virtual
// particles) or recombination photons to emit (rr_on).  Every other tile's
// first forward step would rewrite what it holds.  One thread per tile; the
// whole mark array is rewritten, so no older mark can match.
__global__ __launch_bounds__(256) void k_mark_hop0(const int* __restrict__ rest, const int* __restrict__ head,
                                                   const double* __restrict__ nrr, int rr_on, long long N, int T,
                                                   long long ntiles, int* __restrict__ hot, const long long* cnt,
                                                   int halt_on) {
    if ((halt_on && cnt[kCntHalt] != 0) || cnt[kCntDone] != 0) return;
    const int stamp = static_cast<int>(cnt[kCntSerial]);
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < ntiles; t += (long long)gridDim.x * blockDim.x) {
        bool w = rest[t] != 0;
        const long long j0 = t * T, j1 = (j0 + T < N) ? j0 + T : N;
        for (long long j = j0; j < j1; ++j) w = w || head[j] >= 0 || (rr_on && nrr[j] > 0.0);
        hot[t] = w ? stamp : -1;
    }
}

// The tiles marked for forward step `hop` (tile mark == its stamp), listed with
// their edge ranges for the forward-step kernel: each workgroup takes 4096 marks (16 consecutive per
// thread, read as four 16-byte vectors), a workgroup prefix sum orders its
// marked tiles, and one atomic per workgroup places them.  Within a workgroup
// the list is sorted; workgroups land in any order (the forward step's result
// does not depend on the order it runs tiles in).
__global__ __launch_bounds__(256) void k_tile_list(const int* __restrict__ hot, long long ntiles, int hop, int act_rd,
                                                   const int* __restrict__ rev_off, long long N, int T,
                                                   int4* __restrict__ tlist, long long* cnt, int halt_on) {
    if ((halt_on && cnt[kCntHalt] != 0) || cnt[kCntDone] != 0 || (act_rd >= 0 && cnt[kCntAct0 + kCntLine * act_rd] == 0))
        return;
    list_marked_chunk(hot, ntiles, static_cast<int>(cnt[kCntSerial]) + hop, blockIdx.x, rev_off, N, T, tlist,
                      &cnt[kCntTileList + (hop & 1)]);
}

// Adds the tiles' running tallies of an RT step to the counters and clears them.
// End of a step's forward steps: the per-tile tallies summed, the stamp base
// advanced past the forward steps launched, the step's forward-step count kept.
// graph: the forward steps were a fixed number enqueued in advance; if packets
// are still active after them, the step is left unfinished (halt 1) for the
// host to continue, and nothing is tallied.
__global__ __launch_bounds__(256) void k_step_tally(long long* cnt, unsigned long long* part, long long ntiles,
                                                    long long launched, int graph) {
    __shared__ unsigned long long s[3][256];
    if (graph && cnt[kCntHalt] != 0) return;
    const long long H = cnt[kCntHopsStep];
    if (graph && cnt[kCntAct0 + kCntLine * ((H + 1) & 1)] != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            cnt[kCntHalt] = 1;
            cnt[kCntDone] = 1;  // the forward-step kernel's halt test
        }
        return;
    }
    // the sums first (loads only, so they overlap), then the clears
    unsigned long long v[3] = {0, 0, 0};
#pragma unroll 4
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < ntiles; t += gridDim.x * 256LL)
        for (int c = 0; c < 3; ++c) v[c] += part[3 * t + c];
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < ntiles; t += gridDim.x * 256LL)
        for (int c = 0; c < 3; ++c) part[3 * t + c] = 0;
    for (int c = 0; c < 3; ++c) s[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int c = 0; c < 3; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (s[0][0]) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[kCntUpdates]), s[0][0]);
        if (s[1][0]) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[kCntBytes]), s[1][0]);
        if (s[2][0]) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[kCntTiles]), s[2][0]);
        if (blockIdx.x == 0) {
            cnt[kCntSerial] += launched;
            cnt[kCntLastHops] = H;
        }
    }
}

// Last kernel of a step: an error flag raised by the step halts the steps
// enqueued after it (the host reports it).
__global__ void k_step_end(long long* cnt, int halt_on) {
    if (!halt_on || threadIdx.x != 0 || cnt[kCntHalt] != 0) return;
    if (cnt[kCntFlags] & (kFlagVipOverflow | kFlagRecOverflow | kFlagNonFinite | kFlagDrift)) {
        cnt[kCntHalt] = 2;
        cnt[kCntDone] = 1;  // the forward-step kernel's halt test
    }
}

// ------------------------------------------------------------- chemistry --

struct ChemArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    const long long* cnt;
    long long N;
    int nf, mode, isothermal, freeze, rr_on;
    double dt, frac;
    double* A;
    long long* dep;
    const double* eps;
    const double* nH;
    const double* NH;
    double* xHI;
    double* T;
    double* nrr_wr;
    float* kappa;
    const double* Linst;
    const int* inst_of;
    const double* rc3;  // [N][3] alpha_A, alpha_B, beta at the particle's T while T is
                        // fixed (isothermal or frozen runs), else null
};

// The recombination and collisional-ionization coefficients of each particle
// at its temperature, for runs whose temperatures never change: evaluated once
// instead of every step (the fits' powers and exponentials in FP64 were most
// of the chemistry step), from the same T, hence the same values.
__global__ __launch_bounds__(256) void k_rates_cache(long long N, const double* __restrict__ T, double* __restrict__ rc3) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= N) return;
    const Rates r = rates_at(T[j]);
    rc3[3 * j] = r.aA;
    rc3[3 * j + 1] = r.aB;
    rc3[3 * j + 2] = r.beta;
}

// Chemistry step of one particle (section 2.1; section 2.2 for the RR
// photons).  Gamma = sum_nu A_nu / (N_HI dt) with N_HI at the start of the
// step; the neutral fraction follows dy/dt = alpha n_e (1-y) - (Gamma +
// beta n_e) y by backward Euler over sub-steps that change y by at most
// frac * max(min(y, 1-y), 1e-6) (and T by frac * T); with heating and cooling
// d[(1+x)T]/dt = 2 (H - Lambda) / (3 k n_H), H = n_H y sum_nu Gamma_nu eps_nu
// with the current y.  RR photons: alpha_1 n_e x N_H dt_sub.
__global__ __launch_bounds__(256) void k_chem(ChemArgs a) {
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= a.N) return;
    const double nH = a.nH[j], NH = a.NH[j];
    for (int nu = 0; nu < a.nf; ++nu) {
        long long* d = a.dep + 3 * (j * a.nf + nu);
        if (d[0] != 0 || d[1] != 0 || d[2] != 0) {  // cleared only where something was deposited
            a.A[j * a.nf + nu] += (static_cast<double>(d[0]) * kDepositCoarse + static_cast<double>(d[1]) * kDepositFine +
                                   static_cast<double>(d[2]) * kDepositFiner) * NH;
            d[0] = 0;
            d[1] = 0;
            d[2] = 0;
        }
    }
    double y = a.xHI[j];
    double Tc = a.T[j];
    double rr = 0.0;
    if (a.freeze) {
        if (a.rr_on) {
            Rates rt = {};
            if (a.rc3) {
                rt.aA = a.rc3[3 * j];
                rt.aB = a.rc3[3 * j + 1];
            } else {
                rt = rates_at(Tc);
            }
            const double x = 1.0 - y;
            rr = (rt.aA - rt.aB) * (nH * x) * x * NH * a.dt;
        }
    } else {
        const double nhi0 = y * NH;
        double asum = 0.0, esum = 0.0;
        for (int nu = 0; nu < a.nf; ++nu) {
            asum += a.A[j * a.nf + nu];
            esum += a.A[j * a.nf + nu] * a.eps[nu];
        }
        const double gam = nhi0 > 0.0 ? asum / (nhi0 * a.dt) : 0.0;
        // photoheating per volume n_H y sum_nu Gamma_nu eps_nu, with the current y
        const double heat_y = nhi0 > 0.0 ? esum / (nhi0 * a.dt) * nH : 0.0;
        const bool caseB = a.mode == 0;
        double t = 0.0;
        // isothermal: T, hence every rate coefficient, is fixed over the step
        // (and over the run: the coefficients come from the cache)
        Rates rt = {};
        if (a.rc3) {
            rt.aA = a.rc3[3 * j];
            rt.aB = a.rc3[3 * j + 1];
            rt.beta = a.rc3[3 * j + 2];
        } else {
            rt = rates_at(Tc);
        }
        for (int n = 0; t < a.dt && n < 1000000; ++n) {
            if (!a.isothermal && n > 0) rt = rates_at(Tc);
            const double alpha = caseB ? rt.aB : rt.aA;
            const double x = 1.0 - y;
            const double ne = nH * x;
            const double ion = gam + rt.beta * ne;
            const double rec = alpha * ne;
            const double dydt = rec * x - ion * y;
            double dts = a.dt - t;
            double sc = y < x ? y : x;
            if (sc < 1e-6) sc = 1e-6;
            if (fabs(dydt) > 0.0) {
                const double lim = a.frac * sc / fabs(dydt);
                if (lim < dts) dts = lim;
            }
            double dY = 0.0, Y = 0.0;
            if (!a.isothermal) {
                const double nhi = nH * y, nhii = nH * x;
                const double lam = (caseB ? rt.recB : rt.recA) * ne * nhii + kBoltz * kTHI * rt.beta * ne * nhi +
                                   rt.cexc * ne * nhi + rt.ff * ne * nhii + rt.compton * ne;
                dY = 2.0 * (heat_y * y - lam) / (3.0 * kBoltz * nH);
                Y = (1.0 + x) * Tc;
                if (fabs(dY) > 0.0) {
                    const double limT = a.frac * Y / fabs(dY);
                    if (limT < dts) dts = limT;
                }
            }
            const double yn = (y + dts * rec) / (1.0 + dts * (ion + rec));
            if (a.rr_on) rr += (rt.aA - rt.aB) * ne * (1.0 - yn) * NH * dts;
            if (!a.isothermal) {
                Y = Y + dts * dY;
                Tc = Y / (2.0 - yn);
                if (Tc < 10.0) Tc = 10.0;
            }
            y = yn;
            t += dts;
        }
        a.xHI[j] = y;
        a.T[j] = Tc;
    }
    a.nrr_wr[j] = a.rr_on ? rr : 0.0;
    if (a.kappa) a.kappa[j] = static_cast<float>(y * nH * a.Linst[a.inst_of[j]]);
}

// ---------------------------------------------------------------- ledger --

constexpr int kLedgerBinsPerPass = 4;  // bins summed per pass of k_ledger_partial

struct LedgerArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    const long long* cnt;
    int nf, rr_bin, rr_on;
    long long n_chunks;
    const int* chunk_inst;
    const long long* chunk_lo;
    const long long* chunk_hi;
    const double* A;
    const double* nrr_prev;
    const double* Fp;      // [N][nf] photons resting in the bins (written by the forward steps)
    double* partial;       // [n_chunks][nf][3]: E_rr, A, F
};

// Per chunk of one instance's particles: fixed-order partial sums.
__global__ __launch_bounds__(256) void k_ledger_partial(LedgerArgs a) {
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const long long c = blockIdx.x;
    const long long lo = a.chunk_lo[c], hi = a.chunk_hi[c];
    __shared__ double red[256];
    // passes over the chunk's particles, four bins at a time (the bins of a
    // particle are adjacent in A and Fp, so a pass reads each line once);
    // each thread adds its particles in the same order for every bin, and the
    // tree below is fixed
    for (int nu0 = 0; nu0 < a.nf; nu0 += kLedgerBinsPerPass) {
        double v[kLedgerBinsPerPass][3];
#pragma unroll
        for (int u = 0; u < kLedgerBinsPerPass; ++u) v[u][0] = v[u][1] = v[u][2] = 0.0;
        for (long long j = lo + threadIdx.x; j < hi; j += 256) {
#pragma unroll
            for (int u = 0; u < kLedgerBinsPerPass; ++u) {
                const int nu = nu0 + u;
                if (nu < a.nf) {
                    if (a.rr_on && nu == a.rr_bin) v[u][0] += a.nrr_prev[j];
                    v[u][1] += a.A[j * a.nf + nu];
                    v[u][2] += a.Fp[j * a.nf + nu];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kLedgerBinsPerPass; ++u) {
            const int nu = nu0 + u;
            if (nu >= a.nf) break;
            for (int k = 0; k < 3; ++k) {
                red[threadIdx.x] = v[u][k];
                __syncthreads();
                for (int off = 128; off > 0; off >>= 1) {
                    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
                    __syncthreads();
                }
                if (threadIdx.x == 0) a.partial[(c * a.nf + nu) * 3 + k] = red[0];
                __syncthreads();
            }
        }
    }
}

// Escaped and removed photons of the virtual particles of emission cones,
// summed per instance and bin and cleared for the next step.  One workgroup per
// (instance, bin) runs over that instance's emitters: each lane adds a fixed
// stride of the entries in order and the lanes are combined by a fixed tree, so
// the sums are the same on every run.
constexpr int kEmTallyBlock = 1024;

struct EmitTallyArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    const long long* cnt;
    int nf;
    long long per_em;              // emission cones per emitter and step (sub-steps x N_EC)
    const int* em_by_inst;         // emitter indices grouped by instance
    const long long* em_ioff;      // [n_inst+1] each instance's range in em_by_inst
    double* exs;                   // [emitter][per_em][nf] escaped, cleared here
    double* ers;                   // [emitter][per_em][nf] removed, cleared here
    double* emt;                   // [n_inst][nf][2] escaped, removed
};

__global__ __launch_bounds__(kEmTallyBlock) void k_emit_tally(EmitTallyArgs a) {
    __shared__ double sx[kEmTallyBlock], sr[kEmTallyBlock];
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const int k = blockIdx.x / a.nf, nu = blockIdx.x % a.nf;
    const long long e0 = a.em_ioff[k];
    const long long total = (a.em_ioff[k + 1] - e0) * a.per_em;
    double x = 0.0, r = 0.0;
    for (long long i = threadIdx.x; i < total; i += kEmTallyBlock) {
        const long long m = a.em_by_inst[e0 + i / a.per_em];
        const long long ix = (m * a.per_em + i % a.per_em) * a.nf + nu;
        x += a.exs[ix];
        r += a.ers[ix];
        a.exs[ix] = 0.0;
        a.ers[ix] = 0.0;
    }
    sx[threadIdx.x] = x;
    sr[threadIdx.x] = r;
    __syncthreads();
    for (int w = kEmTallyBlock / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            sx[threadIdx.x] += sx[threadIdx.x + w];
            sr[threadIdx.x] += sr[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.emt[2 * blockIdx.x] = sx[0];
        a.emt[2 * blockIdx.x + 1] = sr[0];
    }
}

struct LedgerFinalArgs {
    int halt_on;  // steps replayed from a graph: exit at once while the halt word is set
    int n_inst, nf, f32;
    const long long* inst_chunk0;   // [n_inst+1] chunk ranges
    const double* partial;          // [n_chunks][nf][3]: E_rr, A, F
    unsigned long long* xr_fx;      // [n_inst][nf][2][3] escaped, removed (fixed point), cleared here
    const double* Ufx;              // [n_inst] their unit
    const double* E_src;            // [n_inst][nf] source photons per step
    const double* emt;              // [n_inst][nf][2] emission-cone escaped, removed (k_emit_tally)
    double* led;                    // [n_inst][nf][5] E, A, X, R, F (F current)
    double* scale;                  // [n_inst][nf]
    long long* cnt;
};

// One workgroup of kLedgerFinalBlock threads per (instance, bin): thread i sums
// the instance's chunks i, i + kLedgerFinalBlock, ... in order, then a fixed
// tree over the threads (the same order on every run, whatever the timing).
constexpr int kLedgerFinalBlock = 256;

__global__ __launch_bounds__(kLedgerFinalBlock) void k_ledger_final(LedgerFinalArgs a) {
    if (a.halt_on && a.cnt[kCntHalt] != 0) return;
    const int t = blockIdx.x;
    if (t >= a.n_inst * a.nf) return;
    const int k = t / a.nf, nu = t % a.nf;
    double v[5] = {0, 0, 0, 0, 0};
    for (long long c = a.inst_chunk0[k] + threadIdx.x; c < a.inst_chunk0[k + 1]; c += kLedgerFinalBlock) {
        v[0] += a.partial[(c * a.nf + nu) * 3 + 0];
        v[1] += a.partial[(c * a.nf + nu) * 3 + 1];
        v[4] += a.partial[(c * a.nf + nu) * 3 + 2];
    }
    __shared__ double s0[kLedgerFinalBlock], s1[kLedgerFinalBlock], s4[kLedgerFinalBlock];
    s0[threadIdx.x] = v[0];
    s1[threadIdx.x] = v[1];
    s4[threadIdx.x] = v[4];
    __syncthreads();
    for (int w = kLedgerFinalBlock / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s4[threadIdx.x] += s4[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    v[0] = s0[0];
    v[1] = s1[0];
    v[4] = s4[0];
    unsigned long long* fx = a.xr_fx + 6 * static_cast<long long>(t);
    v[2] = fx_value3(fx) * a.Ufx[k] + a.emt[2 * t];
    v[3] = fx_value3(fx + 3) * a.Ufx[k] + a.emt[2 * t + 1];
    for (int q = 0; q < 6; ++q) fx[q] = 0ull;
    double* L = a.led + (static_cast<long long>(k) * a.nf + nu) * 5;
    L[0] += a.E_src[k * a.nf + nu] + v[0];
    L[1] += v[1];
    L[2] += v[2];
    L[3] += v[3];
    L[4] = v[4];
    // FP32 transport: the photons in flight are rescaled to what the FP64
    // ledger says is left.  Rounding moves them by ~1e-7 of the photons
    // handled, which can be a large part of few photons in flight, so a
    // difference within 1e-3 of the photons in flight or 1e-5 of those
    // emitted is rounding; anything else (or nothing left to carry) is not
    // rescaled, and reported.
    double s = 1.0;
    if (a.f32 && v[4] > 0.0) {
        const double target = L[0] - L[1] - L[2] - L[3];
        const double diff = fabs(target - v[4]);
        if (target > 0.0 && (diff <= 1e-3 * v[4] || diff <= 1e-5 * L[0]))
            s = target / v[4];
        else
            atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagDrift));
    }
    a.scale[k * a.nf + nu] = s;
    for (int q = 0; q < 5; ++q)
        if (!isfinite(L[q]))
            atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagNonFinite));
}

}  // namespace trt
