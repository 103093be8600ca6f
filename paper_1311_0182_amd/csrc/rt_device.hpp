// rt_device.hpp -- device building blocks of the TRAPHIC step on gfx950:
// counter-based random numbers, rotations, the transmission-cone test, the
// grid-binned k-nearest-neighbour query, the SPH kernel and the rate fits of
// the chemistry.  Everything here runs on the GPU (some helpers are also
// callable on the host for set-up).  Compiled with -ffp-contract=off so that
// the FP64 arithmetic is plain IEEE operations in source order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trt {

constexpr double kCLight = 2.99792458e10;  // cm/s
constexpr double kBoltz = 1.380649e-16;    // erg/K
constexpr double kTHI = 157807.0;          // K, hydrogen ionization potential over k_B
constexpr double kTCMB = 2.725;            // K, CMB temperature today
constexpr int kMaxNgb = 64;
constexpr uint32_t kVipAttempts = 65536;

// Purposes of random draws (first counter word).
enum : uint32_t { kTagRC = 1, kTagEC = 2, kTagVipT = 3, kTagVipE = 4, kTagRREC = 5, kTagVipRR = 6 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies and xors with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint64_t m0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
        const uint64_t m1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
        const uint32_t n0 = static_cast<uint32_t>(m1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(m0 >> 32) ^ c[3] ^ k1;
        c[1] = static_cast<uint32_t>(m1);
        c[3] = static_cast<uint32_t>(m0);
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Four uniforms on (-1, 1), each an exact double (32-bit resolution).
__host__ __device__ inline void uniforms4(uint64_t seed, uint32_t tag, uint32_t attempt,
                                          uint32_t step, uint32_t a, uint32_t b, double u[4]) {
    uint32_t c[4] = {tag | (attempt << 4), step, a, b};
    philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double v = (static_cast<double>(c[i]) + 0.5) * (1.0 / 4294967296.0);
        u[i] = 2.0 * v - 1.0;
    }
}

// Frame of a transmission cone for drawing its points: the unit axis
// a = d/abs(d) and unit vectors e1 = (g x a)/abs(g x a), e2 = a x e1 across it,
// g the coordinate axis least aligned with a (the first of the smallest
// abs(a_k)).  A draw (u0, u1, u2) in [-1, 1)^3 maps to the point
// t a + x e1 + y e2 with t = (u0 + 1)/2, (x, y) = sin(theta) (u1, u2): a box
// that holds the cone's part of the unit ball (about 30% of it is kept,
// against 6.5% of the cube [-1, 1]^3 for N_TC = 8).
struct ConeFrame {
    double a[3], e1[3], e2[3], sn;
};

__host__ __device__ inline ConeFrame cone_frame(const double d[3], double c2) {
    ConeFrame f;
    const double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; ++k) f.a[k] = d[k] / n;
    const double ax = fabs(f.a[0]), ay = fabs(f.a[1]), az = fabs(f.a[2]);
    const int g = (ax <= ay && ax <= az) ? 0 : (ay <= az ? 1 : 2);
    double cr[3];
    if (g == 0) {
        cr[0] = 0.0;
        cr[1] = -f.a[2];
        cr[2] = f.a[1];
    } else if (g == 1) {
        cr[0] = f.a[2];
        cr[1] = 0.0;
        cr[2] = -f.a[0];
    } else {
        cr[0] = -f.a[1];
        cr[1] = f.a[0];
        cr[2] = 0.0;
    }
    const double m = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int k = 0; k < 3; ++k) f.e1[k] = cr[k] / m;
    f.e2[0] = f.a[1] * f.e1[2] - f.a[2] * f.e1[1];
    f.e2[1] = f.a[2] * f.e1[0] - f.a[0] * f.e1[2];
    f.e2[2] = f.a[0] * f.e1[1] - f.a[1] * f.e1[0];
    f.sn = sqrt(1.0 - c2);  // c2 = cos^2(theta), formed as c * c
    return f;
}

__host__ __device__ inline void cone_point(const ConeFrame& f, const double u[4], double p[3]) {
    const double t = 0.5 * (u[0] + 1.0), x = f.sn * u[1], y = f.sn * u[2];
    for (int k = 0; k < 3; ++k) p[k] = t * f.a[k] + x * f.e1[k] + y * f.e2[k];
}

// Haar-uniform rotation: a uniform point of the unit 4-ball (rejection), made
// a unit quaternion, turned into its rotation matrix (row major).
__host__ __device__ inline void random_rotation(uint64_t seed, uint32_t tag, uint32_t step,
                                                uint32_t a, uint32_t b, double R[9]) {
    double q[4];
    double s = 0.0;
    for (uint32_t att = 0;; ++att) {
        uniforms4(seed, tag, att, step, a, b, q);
        s = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (s <= 1.0 && s >= 1e-6) break;
    }
    const double n = sqrt(s);
    const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
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

__host__ __device__ inline void rotate3(const double R[9], const double u[3], double o[3]) {
    o[0] = R[0] * u[0] + R[1] * u[1] + R[2] * u[2];
    o[1] = R[3] * u[0] + R[4] * u[1] + R[5] * u[2];
    o[2] = R[6] * u[0] + R[7] * u[1] + R[8] * u[2];
}

// Transmission cone of solid angle 4 pi / N_TC around d (half-angle with
// cosine C = 1 - 2/N_TC): v.d > 0 and (v.d)^2 >= C^2 |v|^2 |d|^2, inclusive.
template <typename R>
__host__ __device__ inline bool in_cone(R vx, R vy, R vz, R dx, R dy, R dz, R c2) {
    const R a = vx * dx + vy * dy + vz * dz;
    if (!(a > R(0))) return false;
    return a * a >= c2 * (vx * vx + vy * vy + vz * vz) * (dx * dx + dy * dy + dz * dz);
}

// Index of the direction in w[n][3] with the largest dot product with d
// (ties to the lower index): reception-cone binning and Voronoi emission cones.
template <typename R>
__host__ __device__ inline int nearest_direction(const R* w, int n, R dx, R dy, R dz) {
    int best = 0;
    R bv = dx * w[0] + dy * w[1] + dz * w[2];
    for (int k = 1; k < n; ++k) {
        const R v = dx * w[3 * k] + dy * w[3 * k + 1] + dz * w[3 * k + 2];
        if (v > bv) {
            bv = v;
            best = k;
        }
    }
    return best;
}

// The artificial barrier of the shadow test (section 4): a disk of radius r
// around c in the plane x = c_x that removes every photon packet passing
// through it.  A packet passes through it when the straight leg it travels,
// from a to b, meets the disk: the ends not strictly on one side of the plane,
// the leg not in the plane, and the point where it meets the plane within r of
// c (inclusive).  Plain FP64 operations in a fixed order, so the decision is
// the same wherever it is taken.
__host__ __device__ inline bool leg_crosses_disk(const double a[3], const double b[3], const double c[3], double r) {
    const double da = a[0] - c[0], db = b[0] - c[0];
    if ((da > 0.0 && db > 0.0) || (da < 0.0 && db < 0.0)) return false;
    if (da == db) return false;
    const double t = da / (da - db);
    const double py = (a[1] + t * (b[1] - a[1])) - c[1];
    const double pz = (a[2] + t * (b[2] - a[2])) - c[2];
    return py * py + pz * pz <= r * r;
}

// bar: [n_inst][4] centre and radius of each instance's barrier (radius 0:
// none); a null bar when no instance has one
__host__ __device__ inline bool barrier_blocks(const double* bar, int inst, const double a[3], const double b[3]) {
    if (!bar) return false;
    const double* d = bar + 4 * inst;
    return d[3] > 0.0 && leg_crosses_disk(a, b, d, d[3]);
}

// Half-width of the band around a threshold inside which an FP32 decision of
// the transport (cone membership, reception cone) is handed to FP64.  The
// FP32 dot products of unit vectors that decide them are within 1e-6 of the
// exact ones (each operand rounded once: 6e-8; three roundings of the fused
// products: 1.8e-7; lengths within a few ulp of 1: 3e-7), so outside the band
// the FP32 decision is the exact one.
constexpr double kConeGuard = 4e-6;

// nearest_direction for the FP32 transport: the FP32 argmax over the rounded
// directions w32, unless the runner-up lies within kConeGuard of the best; then
// the FP64 argmax over w64 (the FP64 transport's own directions, same rule).
__device__ inline int nearest_direction_guarded(const float* w32, const double* w64, int n, float dx, float dy,
                                                float dz) {
    int best = 0;
    float bv = dx * w32[0] + dy * w32[1] + dz * w32[2];
    float sv = -3.0f;
    for (int k = 1; k < n; ++k) {
        const float v = dx * w32[3 * k] + dy * w32[3 * k + 1] + dz * w32[3 * k + 2];
        if (v > bv) {
            sv = bv;
            bv = v;
            best = k;
        } else if (v > sv) {
            sv = v;
        }
    }
    if (bv - sv < static_cast<float>(kConeGuard))
        best = nearest_direction<double>(w64, n, static_cast<double>(dx), static_cast<double>(dy), static_cast<double>(dz));
    return best;
}

// Absorbed N_in (1 - e^-tau) and transmitted N_in e^-tau parts of a packet leg:
// the smaller part is evaluated directly, the larger is the remainder, so both
// keep full relative precision at any optical depth and they sum to N_in.
template <typename R>
__device__ inline void attenuate(R nin, R tau, R& nabs, R& nout) {
    if (tau < R(0.6931471805599453)) {
        nabs = -nin * expm1(-tau);
        nout = nin - nabs;
    } else {
        nout = nin * exp(-tau);
        nabs = nin - nout;
    }
}

// Cubic-spline kernel shape with support h (Monaghan & Lattanzio 1985); its
// normalisation cancels in normalised interpolation weights.
__device__ inline double spline_shape(double r, double h) {
    const double q = r / h;
    if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) {
        const double t = 1.0 - q;
        return 2.0 * t * t * t;
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// Rate fits (cgs).  Recombination: Hui & Gnedin (1997) case A and B;
// collisional ionization: Hui & Gnedin (1997); cooling: HG97 recombination
// cooling, Cen (1992) collisional excitation, free-free (Gaunt factor 1.3),
// Compton cooling off the z = 0 CMB.
// ---------------------------------------------------------------------------
struct Rates {
    double aA, aB, beta, recA, recB, cexc, ff, compton;
};

__device__ inline Rates rates_at(double T) {
    Rates r;
    const double lam = 2.0 * kTHI / T;
    r.aA = 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
    r.aB = 2.753e-14 * pow(lam, 1.500) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
    r.beta = 21.11 * pow(T, -1.5) * exp(-lam / 2.0) * pow(lam, -1.089) /
             pow(1.0 + pow(lam / 0.354, 0.874), 1.101);
    r.recA = 1.778e-29 * T * pow(lam, 1.965) / pow(1.0 + pow(lam / 0.541, 0.502), 2.697);
    r.recB = 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam / 2.250, 0.376), 3.720);
    r.cexc = 7.5e-19 * exp(-118348.0 / T) / (1.0 + sqrt(T / 1e5));
    r.ff = 1.42e-27 * 1.3 * sqrt(T);
    r.compton = 1.017e-37 * pow(kTCMB, 4.0) * (T - kTCMB);
    return r;
}

// ---------------------------------------------------------------------------
// Uniform cell grid of one instance and the exact k-nearest-neighbour query.
// The result is the N_ngb smallest (d^2, index) pairs, d^2 = (dx dx + dy dy)
// + dz dz with d = x_j - q, which does not depend on the grid.
// ---------------------------------------------------------------------------
struct GridInfo {
    int nc[3];
    int pad;
    double lo[3];
    double cs[3];
    long long cell0;
};

__device__ inline void knn_insert(double* bd, int* bi, int& cnt, int K, double d2, int j) {
    if (cnt == K) {
        const double ld = bd[K - 1];
        if (d2 > ld || (d2 == ld && j > bi[K - 1])) return;
    }
    int pos = (cnt < K) ? cnt++ : K - 1;
    while (pos > 0 && (bd[pos - 1] > d2 || (bd[pos - 1] == d2 && bi[pos - 1] > j))) {
        bd[pos] = bd[pos - 1];
        bi[pos] = bi[pos - 1];
        --pos;
    }
    bd[pos] = d2;
    bi[pos] = j;
}

// Fills bi[0..K) / bd[0..K) sorted ascending; returns h = sqrt(bd[K-1]).
__device__ inline double knn_query(const GridInfo& g, const int* __restrict__ cell_start,
                                   const int* __restrict__ cell_idx, const double* __restrict__ pos,
                                   double qx, double qy, double qz, int self, int K, double* bd,
                                   int* bi) {
    int cnt = 0;
    int c[3];
    const double q[3] = {qx, qy, qz};
    for (int a = 0; a < 3; ++a) {
        int v = static_cast<int>(floor((q[a] - g.lo[a]) / g.cs[a]));
        v = v < 0 ? 0 : (v >= g.nc[a] ? g.nc[a] - 1 : v);
        c[a] = v;
    }
    double csmin = g.cs[0] < g.cs[1] ? g.cs[0] : g.cs[1];
    csmin = csmin < g.cs[2] ? csmin : g.cs[2];
    int smax = g.nc[0] > g.nc[1] ? g.nc[0] : g.nc[1];
    smax = smax > g.nc[2] ? smax : g.nc[2];
    for (int s = 0; s <= smax; ++s) {
        const int x0 = c[0] - s < 0 ? 0 : c[0] - s, x1 = c[0] + s >= g.nc[0] ? g.nc[0] - 1 : c[0] + s;
        const int y0 = c[1] - s < 0 ? 0 : c[1] - s, y1 = c[1] + s >= g.nc[1] ? g.nc[1] - 1 : c[1] + s;
        const int z0 = c[2] - s < 0 ? 0 : c[2] - s, z1 = c[2] + s >= g.nc[2] ? g.nc[2] - 1 : c[2] + s;
        for (int ix = x0; ix <= x1; ++ix) {
            const int ex = abs(ix - c[0]);
            for (int iy = y0; iy <= y1; ++iy) {
                const int exy = max(ex, abs(iy - c[1]));
                for (int iz = z0; iz <= z1; ++iz) {
                    // only the shell at Chebyshev distance s
                    if (max(exy, abs(iz - c[2])) != s) {
                        if (iz < c[2] + s && exy < s) iz = c[2] + s - 1;  // skip the interior
                        continue;
                    }
                    const long long cell = g.cell0 + (static_cast<long long>(ix) * g.nc[1] + iy) * g.nc[2] + iz;
                    const int t1 = cell_start[cell + 1];
                    for (int t = cell_start[cell]; t < t1; ++t) {
                        const int j = cell_idx[t];
                        if (j == self) continue;
                        const double dx = pos[3 * static_cast<long long>(j) + 0] - qx;
                        const double dy = pos[3 * static_cast<long long>(j) + 1] - qy;
                        const double dz = pos[3 * static_cast<long long>(j) + 2] - qz;
                        const double d2 = dx * dx + dy * dy + dz * dz;
                        knn_insert(bd, bi, cnt, K, d2, j);
                    }
                }
            }
        }
        const double reach = static_cast<double>(s) * csmin;
        if (cnt == K && bd[K - 1] <= reach * reach) break;
    }
    return sqrt(bd[K - 1]);
}

// ---------------------------------------------------------------------------
// Wavefront-cooperative exact kNN.  The cube of cells within Chebyshev
// distance 2, then shell by Chebyshev shell, the 64 lanes list the cells with
// their particle ranges (four cells
// per lane per round, loads issued together), a prefix sum over the ranges
// numbers the candidates, and the lanes take four candidates each per round
// (index and position loads issued together), appending (d^2, index) to an
// LDS buffer.  Once there are at least K, the K-th smallest pair in
// (d^2, index) order is found by bisection on the bits of d^2 (non-negative
// doubles order like their bit patterns), counting with one ballot per
// register slot; the search stops when that distance cannot be beaten by
// unvisited cells, and otherwise the buffer is cut to the K best and later
// shells only add candidates no farther than the current K-th.  The same cut
// is made within a pass whenever the next round of candidates might not fit,
// so a dense cube of cells (hundreds of particles around a clustered point)
// stays in the buffer.  Same result as the serial query (the K smallest pairs
// are unique).
// ---------------------------------------------------------------------------
constexpr int kWaveCand = 640;
constexpr int kWavePer = kWaveCand / 64;
constexpr int kWaveCells = 256;

struct WaveKnn {
    double d2[kWaveCand];
    int idx[kWaveCand];
    double res_d2[kMaxNgb];
    int res_idx[kMaxNgb];
    int cfirst[kWaveCells];    // listed cells: first entry in the cell index
    int cpre[kWaveCells + 1];  // prefix sums of their particle counts
    double kth;
    int n;
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Offset of the q-th cell of the Chebyshev shell s (q < number of cells in it).
__device__ inline void shell_cell(int s, int q, int& dx, int& dy, int& dz) {
    if (s == 0) {
        dx = dy = dz = 0;
        return;
    }
    const int side = 2 * s + 1, inner = side - 2;
    const int fa = side * side, fb = side * inner;
    if (q < 2 * fa) {  // the two faces |dz| = s
        const int f = q / fa, m = q - f * fa;
        dz = f ? s : -s;
        dx = m / side - s;
        dy = m - (m / side) * side - s;
    } else if (q < 2 * fa + 2 * fb) {  // |dy| = s, |dz| < s
        const int qq = q - 2 * fa, f = qq / fb, m = qq - f * fb;
        dy = f ? s : -s;
        dx = m / inner - s;
        dz = m - (m / inner) * inner - (s - 1);
    } else {  // |dx| = s, |dy| < s, |dz| < s
        const int fc = inner * inner;
        const int qq = q - 2 * fa - 2 * fb, f = qq / fc, m = qq - f * fc;
        dx = f ? s : -s;
        dy = m / inner - (s - 1);
        dz = m - (m / inner) * inner - (s - 1);
    }
}

// Number of register-held candidates (over the wave) that satisfy pred.
template <typename P>
__device__ inline int wave_count(P pred) {
    int c = 0;
#pragma unroll
    for (int i = 0; i < kWavePer; ++i) c += __popcll(__ballot(pred(i)));
    return c;
}

// The n <= 128 candidates in L.d2/L.idx sorted by (d^2, index) with a
// bitonic network over the wavefront (element e = lane + 64 i in register i):
// the first K of them are exactly the K that the selection below keeps, here
// written back in order to L.d2/L.idx[0..K).  Returns the K-th d^2.
__device__ inline double wave_sort_small(WaveKnn& L, int n, int K, int lane) {
    unsigned long long kd[2];
    int ki[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = lane + 64 * i;
        kd[i] = e < n ? static_cast<unsigned long long>(__double_as_longlong(L.d2[e])) : ~0ull;  // d2 >= 0: ordered as bits
        ki[i] = e < n ? L.idx[e] : 0x7fffffff;
    }
    wave_sync();
    const int top = n <= 64 ? 64 : 128;
    for (int k = 2; k <= top; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j == 64) {
                // partners e and e + 64 sit in the same lane; k = 128 sorts ascending
                const bool sw = kd[1] < kd[0] || (kd[1] == kd[0] && ki[1] < ki[0]);
                if (sw) {
                    const unsigned long long t = kd[0];
                    kd[0] = kd[1];
                    kd[1] = t;
                    const int u = ki[0];
                    ki[0] = ki[1];
                    ki[1] = u;
                }
                continue;
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (i == 1 && top == 64) break;
                const int e = lane + 64 * i;
                const unsigned long long pk = __shfl_xor(kd[i], j, 64);
                const int pi = __shfl_xor(ki[i], j, 64);
                const bool up = (e & k) == 0;       // this block sorts ascending
                const bool low = (lane & j) == 0;   // e is the lower of the pair
                const bool pless = pk < kd[i] || (pk == kd[i] && pi < ki[i]);
                const bool pmore = pk > kd[i] || (pk == kd[i] && pi > ki[i]);
                if (low == up ? pless : pmore) {
                    kd[i] = pk;
                    ki[i] = pi;
                }
            }
        }
    }
    if (lane < K) {
        L.d2[lane] = __longlong_as_double(static_cast<long long>(kd[0]));
        L.idx[lane] = ki[0];
    }
    const double kth = __longlong_as_double(static_cast<long long>(__shfl(kd[0], K - 1, 64)));
    wave_sync();
    return kth;
}

// Selects the K smallest of the n candidates in L.d2/L.idx (K <= n <=
// kWaveCand) and writes them, compacted in arbitrary order, to L.d2/L.idx
// [0, K).  Returns the K-th smallest d^2.
__device__ inline double wave_select(WaveKnn& L, int n, int K, int lane) {
    unsigned long long kb[kWavePer];
    int ki[kWavePer];
#pragma unroll
    for (int i = 0; i < kWavePer; ++i) {
        const int e = i * 64 + lane;
        kb[i] = e < n ? static_cast<unsigned long long>(__double_as_longlong(L.d2[e])) : ~0ull;
        ki[i] = e < n ? L.idx[e] : 0x7fffffff;
    }
    wave_sync();
    // smallest t with #{d2 <= t} >= K
    unsigned long long lo = ~0ull, hi = 0;
#pragma unroll
    for (int i = 0; i < kWavePer; ++i)
        if (kb[i] != ~0ull) {
            lo = kb[i] < lo ? kb[i] : lo;
            hi = kb[i] > hi ? kb[i] : hi;
        }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long ol = __shfl_xor(lo, off, 64), oh = __shfl_xor(hi, off, 64);
        lo = ol < lo ? ol : lo;
        hi = oh > hi ? oh : hi;
    }
    while (lo < hi) {
        const unsigned long long mid = lo + ((hi - lo) >> 1);
        if (wave_count([&](int i) { return kb[i] <= mid; }) >= K)
            hi = mid;
        else
            lo = mid + 1;
    }
    const unsigned long long t = lo;
    const int nlt = wave_count([&](int i) { return kb[i] < t; });
    const int neq = wave_count([&](int i) { return kb[i] == t; });
    // among the pairs at distance t, the (K - nlt) smallest indices
    int umax = 0x7fffffff;
    if (neq > K - nlt) {
        int ulo = 0, uhi = 0x7ffffffe;
        while (ulo < uhi) {
            const int mid = ulo + ((uhi - ulo) >> 1);
            if (wave_count([&](int i) { return kb[i] == t && ki[i] <= mid; }) >= K - nlt)
                uhi = mid;
            else
                ulo = mid + 1;
        }
        umax = ulo;
    }
    int base = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < kWavePer; ++i) {
        const bool sel = kb[i] < t || (kb[i] == t && ki[i] <= umax);
        const unsigned long long b = __ballot(sel);
        if (sel) {
            const int at = base + __popcll(b & below);
            L.d2[at] = __longlong_as_double(static_cast<long long>(kb[i]));
            L.idx[at] = ki[i];
        }
        base += __popcll(b);
    }
    wave_sync();
    return __longlong_as_double(static_cast<long long>(t));
}

// Returns false if the candidate buffer overflowed (the caller then falls
// back to the serial query; with the cuts above this needs K > kWaveCand - 256,
// beyond kMaxNgb, so it is a guard only).  On success res_idx/res_d2[0..K)
// are sorted and kth = res_d2[K-1].
__device__ inline bool knn_wave(const GridInfo& g, const int* __restrict__ cell_start,
                                const int* __restrict__ cell_idx, const double* __restrict__ cpos,
                                double qx, double qy, double qz, int self, int K, WaveKnn& L, int lane) {
    int c[3];
    const double q[3] = {qx, qy, qz};
    for (int a = 0; a < 3; ++a) {
        int v = static_cast<int>(floor((q[a] - g.lo[a]) / g.cs[a]));
        c[a] = v < 0 ? 0 : (v >= g.nc[a] ? g.nc[a] - 1 : v);
    }
    double csmin = g.cs[0] < g.cs[1] ? g.cs[0] : g.cs[1];
    csmin = csmin < g.cs[2] ? csmin : g.cs[2];
    int smax = g.nc[0] > g.nc[1] ? g.nc[0] : g.nc[1];
    smax = smax > g.nc[2] ? smax : g.nc[2];
    const unsigned long long below = (1ull << lane) - 1ull;
    double bound = __longlong_as_double(0x7ff0000000000000ll);  // +inf: keep every candidate
    int n = 0;                                                   // candidates in the buffer
    bool over = false;
    // the first pass takes the whole cube of Chebyshev radius s0 (the usual
    // answer for an interior point), later passes one shell each
    const int s0 = smax < 2 ? smax : 2;
    for (int s = s0; s <= smax; ++s) {
        const bool cube = s == s0;
        const int side = 2 * s + 1;
        const int ncell = cube ? side * side * side : 24 * s * s + 2;  // (2s+1)^3 - (2s-1)^3
        for (int c0 = 0; c0 < ncell; c0 += kWaveCells) {
            // the chunk's cells inside the grid that hold particles
            int first[4], cnt[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int qc = c0 + 64 * i + lane;
                first[i] = 0;
                cnt[i] = 0;
                if (qc < ncell) {
                    int dx, dy, dz;
                    if (cube) {
                        dx = qc / (side * side) - s;
                        dy = (qc / side) % side - s;
                        dz = qc % side - s;
                    } else {
                        shell_cell(s, qc, dx, dy, dz);
                    }
                    const int ix = c[0] + dx, iy = c[1] + dy, iz = c[2] + dz;
                    if (ix >= 0 && ix < g.nc[0] && iy >= 0 && iy < g.nc[1] && iz >= 0 && iz < g.nc[2]) {
                        const long long cell = g.cell0 + (static_cast<long long>(ix) * g.nc[1] + iy) * g.nc[2] + iz;
                        first[i] = cell_start[cell];
                        cnt[i] = cell_start[cell + 1] - first[i];
                    }
                }
            }
            int m = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool ok = cnt[i] > 0;
                const unsigned long long b = __ballot(ok);
                if (ok) L.cfirst[m + __popcll(b & below)] = first[i];
                // counts go through cpre, turned into prefix sums below
                if (ok) L.cpre[m + __popcll(b & below) + 1] = cnt[i];
                m += __popcll(b);
            }
            if (lane == 0) L.cpre[0] = 0;
            wave_sync();
            // inclusive prefix sums of the m counts, 64 at a time
            int carry = 0;
            for (int b0 = 0; b0 < m; b0 += 64) {
                int v = b0 + lane < m ? L.cpre[b0 + lane + 1] : 0;
                for (int off = 1; off < 64; off <<= 1) {
                    const int w = __shfl_up(v, off, 64);
                    if (lane >= off) v += w;
                }
                if (b0 + lane < m) L.cpre[b0 + lane + 1] = v + carry;
                carry += __shfl(v, 63, 64);
            }
            wave_sync();
            const int total = L.cpre[m];
            // the candidates, four per lane per round
            for (int k0 = 0; k0 < total; k0 += 256) {
                // candidate k's entry in cell order: its index and its position
                // (kept in cell order too) load together
                int kc[4], jj[4];
                double d2v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = k0 + 64 * i + lane;
                    kc[i] = -1;
                    if (k < total) {
                        int lo = 0, hi = m - 1;  // the cell holding candidate k
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (L.cpre[mid] <= k)
                                lo = mid;
                            else
                                hi = mid - 1;
                        }
                        kc[i] = L.cfirst[lo] + (k - L.cpre[lo]);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    jj[i] = -1;
                    d2v[i] = 0.0;
                    if (kc[i] >= 0) {
                        jj[i] = cell_idx[kc[i]];
                        const double ex = cpos[3 * static_cast<long long>(kc[i]) + 0] - qx;
                        const double ey = cpos[3 * static_cast<long long>(kc[i]) + 1] - qy;
                        const double ez = cpos[3 * static_cast<long long>(kc[i]) + 2] - qz;
                        d2v[i] = ex * ex + ey * ey + ez * ez;
                    }
                }
                // a full buffer is cut to its K best first (their K-th distance
                // becomes the bound), so a dense cube never overflows it
                if (n + 256 > kWaveCand && n >= K) {
                    bound = wave_select(L, n, K, lane);
                    n = K;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool keep = jj[i] >= 0 && jj[i] != self && d2v[i] <= bound;
                    const unsigned long long b = __ballot(keep);
                    const int at = n + __popcll(b & below);
                    if (keep && at < kWaveCand) {
                        L.d2[at] = d2v[i];
                        L.idx[at] = jj[i];
                    }
                    n += __popcll(b);
                }
            }
            wave_sync();  // the cell lists are reused
            if (n > kWaveCand) over = true;
            if (over) break;
        }
        if (over) return false;
        if (n < K) continue;
        const bool sorted = n <= 128;
        const double kth = sorted ? wave_sort_small(L, n, K, lane) : wave_select(L, n, K, lane);
        const double reach = static_cast<double>(s) * csmin;
        if (kth <= reach * reach || s == smax) {
            // the K selected pairs ordered by (d^2, index)
            if (sorted) {
                if (lane < K) {
                    L.res_d2[lane] = L.d2[lane];
                    L.res_idx[lane] = L.idx[lane];
                }
            } else if (lane < K) {
                const double dc = L.d2[lane];
                const int ic = L.idx[lane];
                int rank = 0;
                for (int u = 0; u < K; ++u) {
                    const double du = L.d2[u];
                    rank += (du < dc) || (du == dc && L.idx[u] < ic);
                }
                L.res_d2[rank] = dc;
                L.res_idx[rank] = ic;
            }
            if (lane == 0) L.kth = kth;
            wave_sync();
            return true;
        }
        bound = kth;
        n = K;
    }
    return true;  // fewer than K particles in the instance
}

}  // namespace trt
