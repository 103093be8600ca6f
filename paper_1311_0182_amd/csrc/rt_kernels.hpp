// rt_kernels.hpp -- gfx950 kernels of one TRAPHIC RT step with recombination
// radiation.  Layout in HBM:
//   packet bins, slot b = (particle j * n_freq + nu) * n_rc + r:
//     pk[b]  = {dx, dy, dz, N}   (Real4; N in photons / U_inst in FP32 mode)
//     pc[b]  = clock              (s in FP64 mode, units of dt in FP32 mode)
//     cm[b]  = bit k set when neighbour k of j lies in the packet's cone
//     sm[b]  = for receiver slot r of (j, nu): bit p set when packet (j, nu, p)
//              moves this forward step and arrives in reception cone r
//   double-buffered (read one, write the other, swap per forward step).
//   Neighbour lists ngb[j*K+k]; reverse lists (receiver-sorted) rev_off /
//   rev_src / rev_pos, each sorted by sender index.
#pragma once

#include "rt_device.hpp"

namespace trt {

// counters in device memory
enum : int {
    kCntSteps = 0,
    kCntHops = 1,
    kCntVips = 2,
    kCntUpdates = 3,
    kCntAct0 = 4,  // active packets for the next forward step, ping-pong [4], [5]
    kCntFlags = 6,
    kCntHopsStep = 7,
    kCntVipCnt0 = 8,  // ViP list fill, ping-pong [8], [9]
    kCntRec = 10,
    kCntDone = 11,    // set once a forward step finds no active packet; later launches of the step exit
    kCntN = 16
};
enum : long long { kFlagHopCap = 1, kFlagVipOverflow = 2, kFlagRecOverflow = 4, kFlagNonFinite = 8 };

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

// Exclusive scan of n ints into out[n+1], one workgroup, sequential chunks.
__global__ __launch_bounds__(1024) void k_scan_i32(const int* __restrict__ in, long long n, int* __restrict__ out) {
    __shared__ int part[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long long base = 0; base < n; base += 1024) {
        const long long i = base + threadIdx.x;
        const int v = i < n ? in[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) out[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_cell_fill(long long N, const int* __restrict__ cell_of, const int* __restrict__ start,
                            int* __restrict__ cursor, int* __restrict__ idx) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int c = cell_of[i];
    idx[start[c] + atomicAdd(&cursor[c], 1)] = static_cast<int>(i);
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

// ---------------------------------------------------------------- per step --

struct StepBeginArgs {
    uint64_t seed;
    uint32_t step;
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
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t == 0) {
        double R[9];
        random_rotation(a.seed, kTagRC, a.step, 0u, 0u, R);
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
        random_rotation(a.seed, kTagEC, a.step, static_cast<uint32_t>(m), static_cast<uint32_t>(sub), R);
        for (int k = 0; k < a.nec; ++k) rotate3(R, a.u_ec + 3 * k, a.ecd + 3 * ((t * a.nec) + k));
    }
}

struct EmitArgs {
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

__device__ inline unsigned long long emis_key(long long m, int sub, int nu, int via, int k, int depth, int arr, int kidx) {
    return (static_cast<unsigned long long>(m) << 37) | (static_cast<unsigned long long>(sub) << 25) |
           (static_cast<unsigned long long>(nu) << 21) | (static_cast<unsigned long long>(via) << 20) |
           (static_cast<unsigned long long>(k) << 12) | (static_cast<unsigned long long>(depth) << 8) |
           (static_cast<unsigned long long>(arr) << 7) | static_cast<unsigned long long>(kidx);
}

// Emission (section 2.1): thread per (emitter, sub-step, neighbour).  Point
// sources: each neighbour belongs to the Voronoi emission cone of the nearest
// rotated direction; a packet is split equally among its cone's members.
// Plane fronts: one packet along +x into the transmission cone.
__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= a.n_emit * a.nsub * a.K) return;
    const int mem = static_cast<int>(t % a.K);
    const long long ms = t / a.K;
    const int sub = static_cast<int>(ms % a.nsub);
    const long long m = ms / a.nsub;
    const int kind = a.em_kind[m];
    if (kind != 0 && sub > 0) return;
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
        for (int u = 0; u < a.K; ++u) {
            const int ju = nb[u];
            const double ux = a.pos[3 * (long long)ju] - ex, uy = a.pos[3 * (long long)ju + 1] - ey, uz = a.pos[3 * (long long)ju + 2] - ez;
            ncone += nearest_direction(E, a.nec, ux, uy, uz) == cone;
        }
        dx = E[3 * cone];
        dy = E[3 * cone + 1];
        dz = E[3 * cone + 2];
        member = true;
    } else {
        member = in_cone(vx, vy, vz, dx, dy, dz, a.c2);
        for (int u = 0; u < a.K; ++u) {
            const int ju = nb[u];
            const double ux = a.pos[3 * (long long)ju] - ex, uy = a.pos[3 * (long long)ju + 1] - ey, uz = a.pos[3 * (long long)ju + 2] - ez;
            ncone += in_cone(ux, uy, uz, dx, dy, dz, a.c2);
        }
    }
    const int r = nearest_direction(a.wrc, a.nrc, dx, dy, dz);
    for (int nu = 0; nu < a.nf; ++nu) {
        const double pk = a.em_pk[m * a.nf + nu];
        if (!(pk > 0.0)) continue;
        if (mem == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntUpdates]),
                                static_cast<unsigned long long>(kind == 0 ? a.nec : 1));
        if (member) {
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
            if (idx >= 0) push_record(a.rec, a.rec_next, a.head, idx, rc);
        }
        // Empty cones become virtual particles (thread mem handles cones mem, mem + K, ...).
        const int nk = kind == 0 ? a.nec : 1;
        for (int kk = mem; kk < nk; kk += a.K) {
            int cntk = 0;
            double kx = 1.0, ky = 0.0, kz = 0.0;
            if (kind == 0) {
                for (int u = 0; u < a.K; ++u) {
                    const int ju = nb[u];
                    const double ux = a.pos[3 * (long long)ju] - ex, uy = a.pos[3 * (long long)ju + 1] - ey, uz = a.pos[3 * (long long)ju + 2] - ez;
                    cntk += nearest_direction(E, a.nec, ux, uy, uz) == kk;
                }
                kx = E[3 * kk];
                ky = E[3 * kk + 1];
                kz = E[3 * kk + 2];
            } else {
                cntk = ncone;
            }
            if (cntk != 0) continue;
            const long long v = push_vip(a.vip, a.cnt, 0, a.vip_cap);
            if (v < 0) continue;
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

struct VipArgs {
    int hop, hop0, max_hops, K, nf, nrc, nec, max_depth;
    uint64_t seed;
    uint32_t step;
    double c2;
    const Vip* list;
    long long vip_cap;
    const double* box;
    const GridInfo* grid;
    const int* cell_start;
    const int* cell_idx;
    const double* pos;
    const double* xHI;
    const double* nH;
    const double* NH;
    const double* sigma;
    const double* wrc;
    const double* ecd;
    double* xs;      // escaped per slot
    double* rs;      // removed per slot
    double* exs;     // escaped per emission packet
    double* ers;     // removed per emission packet
    Rec* rec;
    int* rec_next;
    int* head;
    long long rec_cap;
    long long* cnt;
    int act_rd, act_wr, list_rd, list_wr;
};

// Virtual particles (section 2.1): one thread per packet with an empty cone.
// The particle is drawn uniformly in the cone inside the ball of radius h
// around the origin; outside the box the packet escapes; otherwise it takes
// SPH-interpolated properties from its own neighbours, the leg's absorptions
// go to those neighbours in proportion to W_k N_H,k / n_H,k, and it forwards
// the rest into its own transmission cone (chaining up to max_depth).
__global__ __launch_bounds__(64) void k_vip(VipArgs a) {
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (!a.hop0) {
        // Once one forward step has found nothing to move, every later launch
        // of this step must exit: the ping-pong counters it would read are stale.
        if (a.cnt[kCntDone] != 0 || a.cnt[kCntAct0 + a.act_rd] == 0 || a.hop > a.max_hops) {
            if (gid == 0) a.cnt[kCntDone] = 1;
            return;
        }
    }
    if (gid == 0) {
        a.cnt[kCntAct0 + a.act_wr] = 0;
        a.cnt[kCntVipCnt0 + a.list_wr] = 0;
    }
    long long n = a.cnt[kCntVipCnt0 + a.list_rd];
    if (n > a.vip_cap) n = a.vip_cap;
    double bd[kMaxNgb];
    int bi[kMaxNgb];
    double wk[kMaxNgb];
    for (long long v = gid; v < n; v += (long long)gridDim.x * blockDim.x) {
        Vip q = a.list[v];
        const double* bx = a.box + 6 * q.inst;
        double* X = q.xr_emis ? a.exs : a.xs;
        double* Rm = q.xr_emis ? a.ers : a.rs;
        const GridInfo g = a.grid[q.inst];
        for (int depth = 1;; ++depth) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntVips]), 1ull);
            double p[3] = {0.0, 0.0, 0.0};
            bool ok = false;
            const double* ecs = (q.ec >= 0 && depth == 1) ? a.ecd + 3 * (static_cast<long long>(q.ec) * a.nec) : nullptr;
            for (uint32_t att = 0; att < kVipAttempts; ++att) {
                double u[4];
                uniforms4(a.seed, q.tag, att, a.step, q.ida, q.idb | static_cast<uint32_t>(depth), u);
                p[0] = u[0];
                p[1] = u[1];
                p[2] = u[2];
                if (p[0] * p[0] + p[1] * p[1] + p[2] * p[2] > 1.0) continue;
                if (ecs) {
                    if (nearest_direction(ecs, a.nec, p[0], p[1], p[2]) != q.ek) continue;
                } else if (!in_cone(p[0], p[1], p[2], q.d[0], q.d[1], q.d[2], a.c2)) {
                    continue;
                }
                ok = true;
                break;
            }
            if (!ok) {
                Rm[q.xr] += q.N;
                break;
            }
            const double xv[3] = {q.x[0] + q.h * p[0], q.x[1] + q.h * p[1], q.x[2] + q.h * p[2]};
            if (xv[0] < bx[0] || xv[0] > bx[3] || xv[1] < bx[1] || xv[1] > bx[4] || xv[2] < bx[2] || xv[2] > bx[5]) {
                X[q.xr] += q.N;
                break;
            }
            const double hv = knn_query(g, a.cell_start, a.cell_idx, a.pos, xv[0], xv[1], xv[2], -1, a.K, bd, bi);
            double wsum = 0.0;
            for (int k = 0; k < a.K; ++k) {
                const long long jk = bi[k];
                const double dx = a.pos[3 * jk] - xv[0], dy = a.pos[3 * jk + 1] - xv[1], dz = a.pos[3 * jk + 2] - xv[2];
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                wk[k] = spline_shape(r, hv) * (a.NH[jk] / a.nH[jk]);
                wsum += wk[k];
            }
            if (!(wsum > 0.0)) {
                for (int k = 0; k < a.K; ++k) wk[k] = 1.0;
                wsum = static_cast<double>(a.K);
            }
            double nhi = 0.0;
            for (int k = 0; k < a.K; ++k) nhi += wk[k] * (a.xHI[bi[k]] * a.nH[bi[k]]);
            nhi = nhi / wsum;
            const double dd = sqrt(q.d[0] * q.d[0] + q.d[1] * q.d[1] + q.d[2] * q.d[2]);
            const double l = ((xv[0] - q.x[0]) * q.d[0] + (xv[1] - q.x[1]) * q.d[1] + (xv[2] - q.x[2]) * q.d[2]) / dd;
            const double tau = a.sigma[q.nu] * nhi * l;
            double nabs, nrem;
            attenuate(q.N, tau, nabs, nrem);
            // deposits of the leg's absorptions
            {
                const int idx = alloc_records(a.cnt, a.K, a.rec_cap);
                if (idx >= 0) {
                    for (int k = 0; k < a.K; ++k) {
                        Rec rc;
                        rc.nout = 0.0;
                        rc.dx = rc.dy = rc.dz = 0.0;
                        rc.clk = 0.0;
                        rc.nabs = nabs * wk[k] / wsum;
                        rc.nin = 0.0;
                        rc.key = q.key | (static_cast<unsigned long long>(depth) << 8) | static_cast<unsigned long long>(k);
                        rc.j = bi[k];
                        rc.o = -1 - q.nu;
                        push_record(a.rec, a.rec_next, a.head, idx + k, rc);
                    }
                }
            }
            const double cv = q.c + l / kCLight;
            int nc = 0;
            for (int k = 0; k < a.K; ++k) {
                const long long jk = bi[k];
                nc += in_cone(a.pos[3 * jk] - xv[0], a.pos[3 * jk + 1] - xv[1], a.pos[3 * jk + 2] - xv[2], q.d[0], q.d[1], q.d[2], a.c2);
            }
            if (nc > 0) {
                const int r = nearest_direction(a.wrc, a.nrc, q.d[0], q.d[1], q.d[2]);
                const double nin = nrem / static_cast<double>(nc);
                const int idx = alloc_records(a.cnt, nc, a.rec_cap);
                int w = 0;
                for (int k = 0; k < a.K; ++k) {
                    const long long jk = bi[k];
                    const double vx = a.pos[3 * jk] - xv[0], vy = a.pos[3 * jk + 1] - xv[1], vz = a.pos[3 * jk + 2] - xv[2];
                    if (!in_cone(vx, vy, vz, q.d[0], q.d[1], q.d[2], a.c2)) continue;
                    const double lk = (vx * q.d[0] + vy * q.d[1] + vz * q.d[2]) / dd;
                    const double tk = a.sigma[q.nu] * a.xHI[jk] * a.nH[jk] * lk;
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
                    rc.key = q.key | (static_cast<unsigned long long>(depth) << 8) | (1ull << 7) | static_cast<unsigned long long>(k);
                    rc.j = static_cast<int>(jk);
                    rc.o = q.nu * a.nrc + r;
                    if (idx >= 0) push_record(a.rec, a.rec_next, a.head, idx + w, rc);
                    ++w;
                }
                break;
            }
            if (depth >= a.max_depth) {
                Rm[q.xr] += nrem;
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

template <typename R>
struct HopArgs {
    long long N, B;
    int G, nrc, nf, K, rr_bin, rr_on;
    int hop, hop0, max_hops;
    const double* pos;
    const float4* posf;
    const int* ngb;
    const int* rev_off;
    const int* rev_src;
    const unsigned char* rev_pos;
    const int* inst_of;
    const double* xHI;
    const double* nH;
    const float* kappa;      // FP32: x_HI n_H L_inst
    const R* floor_b;        // floor in bin units
    const double* h;
    const double* sigma;
    const float* sigmaf;
    R c2;
    R dtc;                   // clock limit in clock units
    const float* clf;        // FP32: L_inst / (c dt) per instance
    const double* U;         // photons per bin unit per instance (1 in FP64)
    const double* Linst;     // box side per instance
    const double* scale;     // [n_inst*nf] rescale of in-flight photons at hop 0 (FP32)
    const double* nrr_prev;  // RR photons to emit at hop 0
    const double* wrc;
    const float* wrcf;
    double dt;
    const Bin4<R>* pk_rd;
    const R* pc_rd;
    const unsigned long long* cm_rd;
    const unsigned int* sm_rd;
    Bin4<R>* pk_wr;
    R* pc_wr;
    unsigned long long* cm_wr;
    unsigned int* sm_wr;
    double* A;
    double* P;
    const Rec* rec;
    const int* rec_next;
    const int* head_rd;
    int* head_reset;
    Vip* vip_out;
    long long vip_cap;
    int list_wr;
    long long* cnt;
    int act_rd, act_wr;
};

template <typename R>
struct Acc {
    R n, sx, sy, sz, sc;
    // compensation terms (FP32 only)
    R en, ex, ey, ez, ec;
};

template <typename R>
__device__ inline void tsum(R& s, R& e, R x) {
    // Knuth's TwoSum: s + e accumulates x with its rounding error kept in e.
    const R t = s + x;
    const R z = t - s;
    e += (s - (t - z)) + (x - z);
    s = t;
}

template <typename R>
__device__ inline void acc_add(Acc<R>& a, R n, R dx, R dy, R dz, R c) {
    if constexpr (sizeof(R) == 4) {
        tsum(a.n, a.en, n);
        tsum(a.sx, a.ex, n * dx);
        tsum(a.sy, a.ey, n * dy);
        tsum(a.sz, a.ez, n * dz);
        tsum(a.sc, a.ec, n * c);
    } else {
        a.n += n;
        a.sx += n * dx;
        a.sy += n * dy;
        a.sz += n * dz;
        a.sc += n * c;
    }
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

// One forward step (section 2.1), receiver-sorted: lane = (particle j, bin nu,
// reception cone r).  The lane gathers, over j's incoming neighbour edges,
// the packets that move this step and arrive in its cone (split equally among
// their cone members, attenuated by exp(-tau)), plus packets that stay, plus
// records of emission and virtual particles, and merges them (photons add,
// direction and clock luminosity-weighted).  Then, for the next step, it
// finds its packet's cone members among j's neighbours and its reception cone
// downstream, and publishes them as bit masks.  Hop 0 of a step merges what
// stays (clocks carried over by -dt), the recombination photons of the last
// chemistry step (section 2.2) and the emission records.
template <typename R>
__global__ __launch_bounds__(256) void k_hop(HopArgs<R> a) {
    if (!a.hop0) {
        if (a.cnt[kCntDone] != 0 || a.cnt[kCntAct0 + a.act_rd] == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[kCntDone] = 1;
            return;
        }
        if (a.hop > a.max_hops) {
            if (blockIdx.x == 0 && threadIdx.x == 0)
                atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagHopCap));
            return;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!a.hop0) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntHops]), 1ull);
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntHopsStep]), 1ull);
        }
        a.cnt[kCntRec] = 0;  // records of this step were all linked before launch
    }
    const long long blk = xcd_block(blockIdx.x, gridDim.x);
    const long long s = blk * 256 + threadIdx.x;
    const bool valid = s < a.B;
    const long long j = valid ? s / a.G : 0;
    const int o = valid ? static_cast<int>(s - j * a.G) : 0;
    const int nu = o / a.nrc;
    const int r = o - nu * a.nrc;
    const int inst = valid ? a.inst_of[j] : 0;
    constexpr bool f32 = sizeof(R) == 4;
    const double U = f32 ? a.U[inst] : 1.0;
    const double Linv = f32 ? 1.0 / a.Linst[inst] : 1.0;

    Acc<R> acc = {};
    R asum = 0, aerr = 0, psum = 0, perr = 0;
    bool old_active = false;
    R pjx = 0, pjy = 0, pjz = 0;
    if (valid) {
        if constexpr (f32) {
            const float4 q = a.posf[j];
            pjx = q.x;
            pjy = q.y;
            pjz = q.z;
        } else {
            pjx = a.pos[3 * j];
            pjy = a.pos[3 * j + 1];
            pjz = a.pos[3 * j + 2];
        }
        Bin4<R> q = a.pk_rd[s];
        R c = a.pc_rd[s];
        if (q.n > R(0)) {
            if (a.hop0) {
                if constexpr (f32) q.n = static_cast<R>(static_cast<double>(q.n) * a.scale[inst * a.nf + nu]);
                c = c - a.dtc;
                acc_add(acc, q.n, q.x, q.y, q.z, c);
            } else if (!(c < a.dtc)) {
                acc_add(acc, q.n, q.x, q.y, q.z, c);
            } else {
                old_active = true;
            }
        }
        if (a.hop0 && a.rr_on && nu == a.rr_bin) {
            const double nr = a.nrr_prev[j];
            if (nr > 0.0) {
                const R per = static_cast<R>(nr / static_cast<double>(a.nrc) / U);
                if constexpr (f32)
                    acc_add(acc, per, a.wrcf[3 * r], a.wrcf[3 * r + 1], a.wrcf[3 * r + 2], R(0));
                else
                    acc_add(acc, per, R(a.wrc[3 * r]), R(a.wrc[3 * r + 1]), R(a.wrc[3 * r + 2]), R(0));
            }
        }
        if (!a.hop0) {
            const int e1 = a.rev_off[j + 1];
            R kap = 0, clf = 0, sg = 0;
            if constexpr (f32) {
                kap = a.kappa[j];
                clf = a.clf[inst];
                sg = a.sigmaf[nu];
            }
            for (int e = a.rev_off[j]; e < e1; ++e) {
                const long long i = a.rev_src[e];
                const int kp = a.rev_pos[e];
                const long long base = i * a.G + static_cast<long long>(nu) * a.nrc;
                unsigned int sm = a.sm_rd[base + r];
                if (!sm) continue;
                R vx, vy, vz;
                if constexpr (f32) {
                    // offsets in FP64, rounded once (box units)
                    vx = static_cast<R>((a.pos[3 * j] - a.pos[3 * i]) * Linv);
                    vy = static_cast<R>((a.pos[3 * j + 1] - a.pos[3 * i + 1]) * Linv);
                    vz = static_cast<R>((a.pos[3 * j + 2] - a.pos[3 * i + 2]) * Linv);
                } else {
                    vx = pjx - a.pos[3 * i];
                    vy = pjy - a.pos[3 * i + 1];
                    vz = pjz - a.pos[3 * i + 2];
                }
                while (sm) {
                    const int p = __builtin_ctz(sm);
                    sm &= sm - 1u;
                    const long long t = base + p;
                    const unsigned long long cm = a.cm_rd[t];
                    if (!((cm >> kp) & 1ull)) continue;
                    const Bin4<R> q = a.pk_rd[t];
                    const R ct = a.pc_rd[t];
                    const int nc = __popcll(cm);
                    const R aa = vx * q.x + vy * q.y + vz * q.z;
                    const R l = aa / sqrt(q.x * q.x + q.y * q.y + q.z * q.z);
                    const R nin = q.n / static_cast<R>(nc);
                    R tau, cl;
                    if constexpr (f32) {
                        tau = sg * kap * l;
                        cl = ct + l * clf;
                    } else {
                        tau = a.sigma[nu] * a.xHI[j] * a.nH[j] * l;
                        cl = ct + l / kCLight;
                    }
                    R nabs, nout;
                    attenuate(nin, tau, nabs, nout);
                    sum_add(asum, aerr, nabs);
                    sum_add(psum, perr, nin);
                    acc_add(acc, nout, q.x, q.y, q.z, cl);
                }
            }
        }
        // records of emission and virtual particles, in key order
        const int hd = a.head_rd[j];
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
                last = best;
                first = false;
                sum_add(asum, aerr, static_cast<R>(rc.nabs / U));
                if (rc.o >= 0) {
                    sum_add(psum, perr, static_cast<R>(rc.nin / U));
                    acc_add(acc, static_cast<R>(rc.nout / U), static_cast<R>(rc.dx), static_cast<R>(rc.dy),
                            static_cast<R>(rc.dz), static_cast<R>(f32 ? rc.clk / a.dt : rc.clk));
                }
            }
        }
    }
    // merged packet
    R nn = acc.n + acc.en, sx = acc.sx + acc.ex, sy = acc.sy + acc.ey, sz = acc.sz + acc.ez, sc = acc.sc + acc.ec;
    R dx = 0, dy = 0, dz = 0, cn = 0;
    if (nn > R(0)) {
        const R s2 = sx * sx + sy * sy + sz * sz;
        if (s2 > R(0)) {
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
        cn = sc / nn;
    } else {
        nn = 0;
    }
    if (valid && nn > R(0) && nn < a.floor_b[j]) {
        sum_add(asum, aerr, nn);
        nn = 0;
        dx = dy = dz = cn = 0;
    }
    // absorbed / passing photons of (j, nu): sum over the n_rc lanes
    const R ag = group_sum(asum + aerr, a.nrc);
    const R pg = group_sum(psum + perr, a.nrc);
    if (valid && r == 0) {
        const long long ia = j * a.nf + nu;
        a.A[ia] += static_cast<double>(ag) * U;
        a.P[ia] += static_cast<double>(pg) * U;
    }
    // next forward step: cone members and downstream reception cone
    const bool act = valid && nn > R(0) && cn < a.dtc;
    unsigned long long cmw = 0;
    int tgt = 0;
    if (act) {
        const int* nb = a.ngb + j * a.K;
        const R c2 = a.c2;
        for (int k = 0; k < a.K; ++k) {
            const long long jj = nb[k];
            R vx, vy, vz;
            if constexpr (f32) {
                vx = static_cast<R>((a.pos[3 * jj] - a.pos[3 * j]) * Linv);
                vy = static_cast<R>((a.pos[3 * jj + 1] - a.pos[3 * j + 1]) * Linv);
                vz = static_cast<R>((a.pos[3 * jj + 2] - a.pos[3 * j + 2]) * Linv);
            } else {
                vx = a.pos[3 * jj] - pjx;
                vy = a.pos[3 * jj + 1] - pjy;
                vz = a.pos[3 * jj + 2] - pjz;
            }
            if (in_cone(vx, vy, vz, dx, dy, dz, c2)) cmw |= 1ull << k;
        }
        if constexpr (f32)
            tgt = nearest_direction(a.wrcf, a.nrc, dx, dy, dz);
        else
            tgt = nearest_direction(a.wrc, a.nrc, dx, dy, dz);
    }
    const bool send = act && cmw != 0;
    const bool vip = act && cmw == 0;
    // sender masks: lane r of group (j, nu) gets the packets of the group that go to cone r
    const int lane = threadIdx.x & 63;
    const int gbase = lane & ~(a.nrc - 1);
    const unsigned long long gmask = a.nrc >= 64 ? ~0ull : ((1ull << a.nrc) - 1ull);
    unsigned int mym = 0;
    for (int q = 0; q < a.nrc; ++q) {
        const unsigned long long b = __ballot(send && tgt == q);
        if (r == q) mym = static_cast<unsigned int>((b >> gbase) & gmask);
    }
    if (valid) {
        Bin4<R> w;
        w.x = dx;
        w.y = dy;
        w.z = dz;
        w.n = nn;
        a.pk_wr[s] = w;
        a.pc_wr[s] = cn;
        a.cm_wr[s] = cmw;
        a.sm_wr[s] = mym;
        if (o == 0) a.head_reset[j] = -1;
        if (vip) {
            const long long v = push_vip(a.vip_out, a.cnt, a.list_wr, a.vip_cap);
            if (v >= 0) {
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
    // counters: packets active next step, packets moved this step
    const unsigned long long nact = __popcll(__ballot(act));
    const unsigned long long nupd = __popcll(__ballot(old_active));
    if (lane == 0) {
        if (nact) atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntAct0 + a.act_wr]), nact);
        if (nupd) atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt[kCntUpdates]), nupd);
    }
}

// ------------------------------------------------------------- chemistry --

struct ChemArgs {
    long long N;
    int nf, mode, isothermal, freeze, rr_on;
    double dt, frac;
    const double* A;
    const double* eps;
    const double* nH;
    const double* NH;
    double* xHI;
    double* T;
    double* nrr_wr;
    float* kappa;
    const double* Linst;
    const int* inst_of;
};

// Chemistry step of one particle (section 2.1; section 2.2 for the RR
// photons).  Gamma = sum_nu A_nu / (N_HI dt) with N_HI at the start of the
// step; the neutral fraction follows dy/dt = alpha n_e (1-y) - (Gamma +
// beta n_e) y by backward Euler over sub-steps that change y by at most
// frac * max(min(y, 1-y), 1e-6) (and T by frac * T); with heating and cooling
// d[(1+x)T]/dt = 2 (H - Lambda) / (3 k n_H).  RR photons: alpha_1 n_e x N_H dt_sub.
__global__ __launch_bounds__(256) void k_chem(ChemArgs a) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= a.N) return;
    const double nH = a.nH[j], NH = a.NH[j];
    double y = a.xHI[j];
    double Tc = a.T[j];
    double rr = 0.0;
    if (a.freeze) {
        if (a.rr_on) {
            const Rates rt = rates_at(Tc);
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
        const double heat = esum / ((NH / nH) * a.dt);
        const bool caseB = a.mode == 0;
        double t = 0.0;
        for (int n = 0; t < a.dt && n < 1000000; ++n) {
            const Rates rt = rates_at(Tc);
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
                dY = 2.0 * (heat - lam) / (3.0 * kBoltz * nH);
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

struct LedgerArgs {
    int nf, nrc, G, rr_bin, rr_on, f32;
    long long n_chunks;
    const int* chunk_inst;
    const long long* chunk_lo;
    const long long* chunk_hi;
    const double* A;
    const double* nrr_prev;
    double* xs;
    double* rs;
    const void* pk;        // current bins
    const double* U;
    double* partial;       // [n_chunks][nf][5]: E_rr, A, X, R, F
};

// Per chunk of one instance's particles: fixed-order partial sums.
__global__ __launch_bounds__(256) void k_ledger_partial(LedgerArgs a) {
    const long long c = blockIdx.x;
    const long long lo = a.chunk_lo[c], hi = a.chunk_hi[c];
    const int inst = a.chunk_inst[c];
    const double U = a.f32 ? a.U[inst] : 1.0;
    __shared__ double red[256];
    for (int nu = 0; nu < a.nf; ++nu) {
        double v[5] = {0, 0, 0, 0, 0};
        for (long long j = lo + threadIdx.x; j < hi; j += 256) {
            if (a.rr_on && nu == a.rr_bin) v[0] += a.nrr_prev[j];
            v[1] += a.A[j * a.nf + nu];
            for (int q = 0; q < a.nrc; ++q) {
                const long long b = j * a.G + static_cast<long long>(nu) * a.nrc + q;
                v[2] += a.xs[b];
                v[3] += a.rs[b];
                a.xs[b] = 0.0;
                a.rs[b] = 0.0;
                if (a.f32)
                    v[4] += static_cast<double>(static_cast<const Bin4<float>*>(a.pk)[b].n) * U;
                else
                    v[4] += static_cast<const Bin4<double>*>(a.pk)[b].n;
            }
        }
        for (int k = 0; k < 5; ++k) {
            red[threadIdx.x] = v[k];
            __syncthreads();
            for (int off = 128; off > 0; off >>= 1) {
                if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
                __syncthreads();
            }
            if (threadIdx.x == 0) a.partial[(c * a.nf + nu) * 5 + k] = red[0];
            __syncthreads();
        }
    }
}

struct LedgerFinalArgs {
    int n_inst, nf, f32, nec, nsub;
    long long n_emit;
    const long long* inst_chunk0;   // [n_inst+1] chunk ranges
    const double* partial;
    const double* E_src;            // [n_inst][nf] source photons per step
    const int* em_inst;
    double* exs;
    double* ers;
    double* led;                    // [n_inst][nf][5] E, A, X, R, F (F current)
    double* scale;                  // [n_inst][nf]
    long long* cnt;
};

__global__ void k_ledger_final(LedgerFinalArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_inst * a.nf) return;
    const int k = t / a.nf, nu = t % a.nf;
    double v[5] = {0, 0, 0, 0, 0};
    for (long long c = a.inst_chunk0[k]; c < a.inst_chunk0[k + 1]; ++c)
        for (int q = 0; q < 5; ++q) v[q] += a.partial[(c * a.nf + nu) * 5 + q];
    const long long per_em = static_cast<long long>(a.nsub) * a.nec;
    for (long long m = 0; m < a.n_emit; ++m) {
        if (a.em_inst[m] != k) continue;
        for (long long u = 0; u < per_em; ++u) {
            const long long ix = (m * per_em + u) * a.nf + nu;
            v[2] += a.exs[ix];
            v[3] += a.ers[ix];
            a.exs[ix] = 0.0;
            a.ers[ix] = 0.0;
        }
    }
    double* L = a.led + (static_cast<long long>(k) * a.nf + nu) * 5;
    L[0] += a.E_src[k * a.nf + nu] + v[0];
    L[1] += v[1];
    L[2] += v[2];
    L[3] += v[3];
    L[4] = v[4];
    double s = 1.0;
    if (a.f32 && v[4] > 0.0) {
        const double target = L[0] - L[1] - L[2] - L[3];
        if (fabs(target - v[4]) <= 1e-3 * v[4]) s = target / v[4];
    }
    a.scale[k * a.nf + nu] = s;
    for (int q = 0; q < 5; ++q)
        if (!isfinite(L[q]))
            atomicOr(reinterpret_cast<unsigned long long*>(&a.cnt[kCntFlags]), static_cast<unsigned long long>(kFlagNonFinite));
}

}  // namespace trt
