// traphic_rt.hip -- host side of the MI355X TRAPHIC library: context, device
// memory, the C ABI of include/traphic_rt.h and the launch sequence of a step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/traphic_rt.h"
#include "rt_kernels.hpp"
#include "rt_profile.hpp"

using namespace trt;

namespace {

constexpr int kChunk = 2048;      // particles per ledger partial sum
constexpr int kCellDense = 8;     // particles in the fullest neighbour-search cell before cells are refined
constexpr int kMaxDevices = 64;
// Scratch of rt_shell_profile_noalloc: the shell histogram (sums, then
// counts), the largest any call may need.
constexpr size_t kProfScratchBytes = sizeof(double) * kProfMaxCells + sizeof(unsigned long long) * kProfMaxShells;

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
};

}  // namespace

// Allocation-free scratch (rt_shell_profile_noalloc): one copy per GPU, held
// until the process ends.  Host code never uses this name as an address: the
// device address of each GPU's copy is looked up once per device and kept in
// g_scratch.
static __device__ __align__(256) unsigned char scratch[kProfScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

// The tuner times the configurations with one tile per workgroup.  Packing
// up to four tiles per workgroup cut the dispatch of workgroups with nothing
// to do while every forward step dispatched one per tile; with grids sized
// from the lists, packing only lowers the occupancy that LDS allows (measured
// slower on the batched HII regions and the 64^3 Stromgren sphere once the
// lists reach their working size,
// though not in the first RT steps, where the tuner would see them), so the
// packed configurations are used only when asked for.
constexpr int kTuneShapes = kHopShapeKinds;

struct rt_ctx {
    rt_params p{};
    hipStream_t stream = nullptr;
    int dev = 0;           // device current at rt_init (the stream's)
    bool sticky = false;
    std::string err;

    long long N = 0, B = 0;
    int n_inst = 0, G = 0, nf = 0, K = 0, nrc = 0, nec = 0, nsub = 1;
    bool f32 = false, rr_on = false, rr_orig = false;  // RR photons produced; predecessor scheme
    double c2 = 0.0;
    std::vector<long long> inst_off;
    std::vector<double> box, sigma, eps, U, L;
    std::vector<DevBuf> owned;

    // static geometry
    int* inst_of = nullptr;
    double* box_d = nullptr;
    double* pos = nullptr;
    double *nH = nullptr, *NH = nullptr, *xHI = nullptr, *T = nullptr, *h = nullptr;
    void* floor_b = nullptr;
    float* kappa = nullptr;
    double* sigma_d = nullptr;
    float* sigmaf_d = nullptr;
    double* eps_d = nullptr;
    double* U_d = nullptr;
    double* L_d = nullptr;
    float* clf_d = nullptr;
    int* ngb = nullptr;
    int* rev_off = nullptr;
    int* rev_src = nullptr;
    unsigned char* rev_pos = nullptr;
    GridInfo* grid_d = nullptr;
    int* cell_start = nullptr;
    int* cell_idx = nullptr;
    double* cell_pos = nullptr;  // positions in cell order (cell_idx order), for the wavefront kNN
    int* scan_tmp = nullptr;     // block sums and their offsets of the many-workgroup scan
    double *u_rc = nullptr, *u_ec = nullptr;
    double* rot = nullptr;
    float* wrcf = nullptr;
    // emitters
    long long n_emit = 0;
    int* em_kind = nullptr;
    int* em_inst = nullptr;
    double* em_pos = nullptr;
    double* em_pk = nullptr;
    int* em_ngb = nullptr;
    double* em_h = nullptr;
    double* ecd = nullptr;
    double* exs = nullptr;
    double* ers = nullptr;
    std::vector<int> h_em_inst;
    int* em_by_inst = nullptr;      // emitter indices grouped by instance
    long long* em_ioff = nullptr;   // [n_inst+1] ranges in em_by_inst
    double* emt = nullptr;          // [n_inst][nf][2] emission-cone escaped, removed per step
    double* E_src = nullptr;
    // intensity profiles: histogram and an optional copy of caller-given passing photons
    double* prof_sum = nullptr;
    unsigned long long* prof_cnt = nullptr;
    double* prof_in = nullptr;
    // dynamic state: resting packets (in place), moving packets and delivery
    // masks (by forward-step parity), work marks of the tiles
    void* pk = nullptr;
    void* pcl = nullptr;
    unsigned long long* cm = nullptr;
    void* mv[2] = {nullptr, nullptr};
    void* mvc[2] = {nullptr, nullptr};
    void* inbox[2] = {nullptr, nullptr};
    int* hot[2] = {nullptr, nullptr};
    double* rc3 = nullptr;  // [N][3] rate coefficients while T never changes (isothermal or frozen)
    int* rest = nullptr;    // per tile: photons rest in its bins (left by its last run)
    bool rest_unknown = true;  // rest is all ones (set up or restored): hop 0's next list is every tile
    bool list0 = true;      // hop 0 runs a list of tiles (not with the predecessor RR scheme)
    int4* tlist = nullptr;  // tiles marked for the next forward step, with their edge ranges
    long long hot_len = 0; // entries of each mark array: ntiles padded to whole k_tile_list chunks
    unsigned long long* part = nullptr;  // per-tile tallies of a forward step
    unsigned int* rev_ik = nullptr;
    void* rev_v = nullptr;
    void* fwd_v = nullptr;
    int tileT = 1;         // particles per forward-step workgroup (a power of two)
    int lgT = 0;
    long long ntiles = 0;
    size_t inbox_bytes = 0;
    bool dl64 = false;     // delivery masks need 64 bits (N_RC * N_freq > 32)
    long long serial = 0;  // stamp of hop 0 of the next RT step
    long long last_stamp = -1;  // stamp of the last forward step that ran
    double *A = nullptr, *P = nullptr;
    long long* dep = nullptr;  // fixed-point deposits of virtual particles
    double* nrr[2] = {nullptr, nullptr};
    int nrr_cur = 0;
    double* Fp = nullptr;                 // [N][nf] photons resting in the bins
    unsigned long long* xr_fx = nullptr;  // [n_inst][nf][2][3] escaped, removed (fixed point)
    double* Ufx = nullptr;                // [n_inst] mean N_H: unit of xr_fx
    double* bar_d = nullptr;              // [n_inst][4] barrier disks (radius 0: none)
    // predecessor RR scheme: rotated directions per particle and sub-step,
    // per edge and sub-step the leg's photons and cell, per slot of the RR bin
    // the arrivals' sums
    double* rr_ecd = nullptr;
    double* rr_share = nullptr;
    unsigned char* rr_cone = nullptr;
    double* rr_pre = nullptr;
    std::vector<double> bar;              // host copy
    bool any_bar = false;                 // some instance has a barrier
    Vip* vip[2] = {nullptr, nullptr};
    Vip* deep = nullptr;        // chains that landed inside their box, and their points
    double* deep_x = nullptr;
    long long vip_cap = 0;
    Rec* rec = nullptr;
    int* rec_next = nullptr;
    int* head[2] = {nullptr, nullptr};
    long long rec_cap = 0;
    long long* cnt = nullptr;
    long long* h_cnt = nullptr;  // pinned host mirror
    double* led = nullptr;
    double* scale = nullptr;
    double* partial = nullptr;
    long long n_chunks = 0;
    int* chunk_inst = nullptr;
    long long* chunk_lo = nullptr;
    long long* chunk_hi = nullptr;
    long long* inst_chunk0 = nullptr;
    long long step = 0;
    long long last_hops = 8;   // forward steps of the previous RT step
    // forward steps 1..n of an RT step, captured once per n and replayed
    std::map<int, hipGraphExec_t> hop_graphs;
    std::map<long long, hipGraphExec_t> step_graphs;  // whole RT steps, by 2 * forward steps + RR buffer parity
    bool step_graphs_on = false;                      // rt_set_step_graphs
    bool capturing = false;                           // a whole step is being captured: its kernels obey the halt word
    // forward-step grids: the longest tile list seen per forward step index,
    // from the device's record of each step's lists
    int* listlen = nullptr;
    int* h_listlen = nullptr;                         // pinned copy
    std::vector<long long> est_tiles;
    std::vector<long long> cap_tiles;                 // tiles the main grid of each forward step covered
    // autotuner of the forward-step shape: -1 tune once work is representative
    int hop_shape = 0;
    int tune_mode = -1;        // -1 automatic, -2 tune now, 0..kHopShapes-1 fixed by the caller
    int tune_steps_left = kTuneShapes;  // RT steps that time the shapes (alternating per forward step)
    double tune_ms[kHopShapes] = {};
    long long tune_n[kHopShapes] = {};
    bool tuned = false;
    bool tuning_now = false;   // this RT step times the shapes
    bool graphs_ok = true;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double tm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace {

rt_status fail(rt_ctx* c, rt_status s, const std::string& m) {
    if (c) {
        c->err = m;
        if (s == RT_EDEVICE) c->sticky = true;
    }
    return s;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, RT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// The device address of this process's scratch on the context's GPU, looked
// up once per device with that device current (rt_init does it; a context
// made before another device's lookup finds its own entry already filled).
rt_status resolve_scratch(rt_ctx* c) {
    if (c->dev < 0 || c->dev >= kMaxDevices) return fail(c, RT_EDEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[c->dev]) return RT_OK;
    int cur = -1;
    HIPCHK(c, hipGetDevice(&cur));
    if (cur != c->dev) HIPCHK(c, hipSetDevice(c->dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != c->dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
        return fail(c, RT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[c->dev] = ptr;
    return RT_OK;
}

rt_status dalloc(rt_ctx* c, void** out, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    void* q = nullptr;
    if (c->p.alloc) {
        q = c->p.alloc(c->p.alloc_user, bytes);
        if (!q) return fail(c, RT_ENOMEM, "allocator callback returned NULL");
    } else {
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return fail(c, RT_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    c->owned.push_back({q, bytes});
    *out = q;
    return RT_OK;
}

// Free a buffer this context allocated (no-op for NULL).  Only once no queued
// work or captured graph refers to it.
template <typename T>
void dfree(rt_ctx* c, T*& p) {
    if (!p) return;
    void* q = const_cast<void*>(static_cast<const void*>(p));
    for (size_t k = 0; k < c->owned.size(); ++k)
        if (c->owned[k].p == q) {
            if (c->p.dealloc)
                c->p.dealloc(c->p.alloc_user, q);
            else if (!c->p.alloc)
                (void)hipFree(q);
            c->owned.erase(c->owned.begin() + static_cast<long>(k));
            break;
        }
    p = nullptr;
}

template <typename T>
rt_status alloc_n(rt_ctx* c, T** out, long long n) {
    return dalloc(c, reinterpret_cast<void**>(out), sizeof(T) * static_cast<size_t>(std::max<long long>(n, 1)));
}

template <typename T>
rt_status upload(rt_ctx* c, T** out, const T* host, long long n) {
    rt_status s = alloc_n(c, out, n);
    if (s != RT_OK) return s;
    if (n > 0) HIPCHK(c, hipMemcpyAsync(*out, host, sizeof(T) * n, hipMemcpyHostToDevice, c->stream));
    return RT_OK;
}

unsigned grid_for(long long n, int bs) { return static_cast<unsigned>(std::max<long long>(1, (n + bs - 1) / bs)); }

// Isotropic direction sets: the cube diagonals for 8, otherwise a spherical
// Fibonacci lattice on one hemisphere mirrored through the centre.
void direction_set(int n, std::vector<double>& u) {
    u.assign(3 * n, 0.0);
    if (n == 8) {
        const double s = 1.0 / std::sqrt(3.0);
        for (int k = 0; k < 8; ++k) {
            u[3 * k + 0] = (k & 4) ? -s : s;
            u[3 * k + 1] = (k & 2) ? -s : s;
            u[3 * k + 2] = (k & 1) ? -s : s;
        }
        return;
    }
    const double ga = M_PI * (3.0 - std::sqrt(5.0));
    const int half = (n % 2 == 0) ? n / 2 : n;
    for (int k = 0; k < half; ++k) {
        const double z = 1.0 - (2.0 * k + 1.0) / static_cast<double>(n);
        const double r = std::sqrt(1.0 - z * z);
        const double ph = ga * static_cast<double>(k);
        u[3 * k + 0] = r * std::cos(ph);
        u[3 * k + 1] = r * std::sin(ph);
        u[3 * k + 2] = z;
    }
    for (int k = half; k < n; ++k)
        for (int a = 0; a < 3; ++a) u[3 * k + a] = -u[3 * (k - half) + a];
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

constexpr long long kHopMinSavedWGs = 65536;
constexpr long long kHopHeadroomTiles = 4096;
constexpr long long kHopTailMinWGs = 256;
constexpr long long kHopTailMaxWGs = 65536;
constexpr long long kHopUnseenWGs = 1024;
constexpr long long kHopUnseenTailWGs = 8192;

// Workgroups for a forward step whose list has had up to `tiles` tiles: a
// quarter more, rounded up to a power of two (so that graphs captured with it
// stay valid while the lists grow a little), at least 64.
long long grid_estimate(long long tiles, int wpb) {
    const long long room = std::max(tiles / 4, kHopHeadroomTiles);
    const long long want = (tiles + room + wpb - 1) / wpb + 1;
    long long g = 64;
    while (g < want) g <<= 1;
    return g;
}

// The grids of forward step `hop` (hop 0 without its list runs every tile) with `wpb`
// tiles per workgroup, for a forward step whose list has had up to `est`
// tiles (0: none seen, for this or any nearby forward step): k_hop's workgroups, returned, and k_hop_tail's in
// *n_tail (0: no tail).  The tail's grid is a 64th of the main one and at
// least a 256th of the full grid and kHopTailMinWGs (a list that outgrows its
// estimate, as the lists of a front advancing step by step do, then still
// fills the chip, while a tail with nothing to do dispatches few workgroups),
// kHopUnseenTailWGs for a forward step not seen yet.  A smaller grid pays only when it saves more workgroups
// than the tail's launch costs (an idle workgroup costs well under a
// nanosecond here, a launch a few microseconds): else the full grid, no tail.
long long hop_grid(const rt_ctx* c, int hop, long long est, int wpb, long long* n_tail) {
    const long long n_full = (c->ntiles + wpb - 1) / wpb;
    *n_tail = 0;
    if (hop == 0 && !c->list0) return n_full;
    const long long n_wg = std::min(n_full, est > 0 ? grid_estimate(est, wpb) : kHopUnseenWGs);
    if (n_full - n_wg < kHopMinSavedWGs) return n_full;
    const long long t = est > 0 ? std::min(kHopTailMaxWGs, std::max(std::max(kHopTailMinWGs, n_full / 256), n_wg / 64))
                                : kHopUnseenTailWGs;
    *n_tail = std::min(n_full - n_wg, t);
    return n_wg;
}

template <typename R, typename DT, typename S, bool kBar>
rt_status launch_hop(rt_ctx* c, int hop, bool pack) {
    HopArgs<R, DT> a{};
    a.N = c->N;
    a.G = c->G;
    a.nrc = c->nrc;
    a.nf = c->nf;
    a.K = c->K;
    a.T = c->tileT;
    a.rr_bin = c->p.rr_bin;
    a.rr_on = c->rr_on && !c->rr_orig ? 1 : 0;  // into the reception cones
    a.rr_pre = c->rr_orig ? c->rr_pre : nullptr;
    a.hop = hop;
    a.hop0 = hop == 0;
    a.list0 = (hop == 0 && c->list0) ? 1 : 0;
    a.rest = c->rest;
    a.max_hops = c->p.max_hops;
    a.pos = c->pos;
    a.rev_off = c->rev_off;
    a.rev_ik = c->rev_ik;
    a.rev_v = c->rev_v;
    a.fwd_v = c->fwd_v;
    a.inst_of = c->inst_of;
    a.xHI = c->xHI;
    a.nH = c->nH;
    a.kappa = c->kappa;
    a.floor_b = static_cast<const R*>(c->floor_b);
    a.h = c->h;
    a.sigma = c->sigma_d;
    a.sigmaf = c->sigmaf_d;
    a.c2 = static_cast<R>(c->c2);
    a.c2d = c->c2;
    {
        const double cc = 1.0 - 2.0 / static_cast<double>(c->p.n_tc);
        a.cos_lo = static_cast<float>(cc - kConeGuard);
        a.cos_hi = static_cast<float>(cc + kConeGuard);
    }
    a.dtc = c->f32 ? R(1) : static_cast<R>(c->p.dt);
    a.clf = c->clf_d;
    a.U = c->U_d;
    a.scale = c->scale;
    a.nrr_prev = c->nrr[c->nrr_cur];
    a.wrc = c->rot + 9;
    a.wrcf = c->wrcf;
    a.dt = c->p.dt;
    a.lgT = c->lgT;
    a.ngb = c->ngb;
    const int rd = (hop + 1) & 1, wr = hop & 1;
    a.pk = static_cast<Bin4<R>*>(c->pk);
    a.pcl = static_cast<R*>(c->pcl);
    a.cm = c->cm;
    a.mv_rd = static_cast<const Bin4<R>*>(c->mv[rd]);
    a.mvc_rd = static_cast<const R2<R>*>(c->mvc[rd]);
    a.in_rd = static_cast<const Inbox<DT>*>(c->inbox[rd]);
    a.hot_rd = c->hot[hop & 1];
    a.tlist = c->tlist;
    a.ntiles = c->ntiles;
    a.mv_wr = static_cast<Bin4<R>*>(c->mv[wr]);
    a.mvc_wr = static_cast<R2<R>*>(c->mvc[wr]);
    a.in_wr = static_cast<Inbox<DT>*>(c->inbox[wr]);
    a.hot_wr = c->hot[(hop + 1) & 1];
    a.A = c->A;
    a.P = c->P;
    a.Fp = c->Fp;
    a.xr_fx = c->xr_fx;
    a.Ufx = c->Ufx;
    a.rec = c->rec;
    a.rec_next = c->rec_next;
    a.head = c->head[hop & 1];
    a.vip_out = c->vip[(hop + 1) & 1];
    a.vip_cap = c->vip_cap;
    a.list_wr = (hop + 1) & 1;
    a.cnt = c->cnt;
    a.part = c->part;
    a.listlen = c->listlen;
    a.act_rd = hop & 1;
    a.act_wr = (hop + 1) & 1;
    // 1, 2 or 4 tiles (wavefronts) per workgroup, as many as 64 KiB of LDS hold
    const size_t lds_wave = (HopLds<R, DT, S>::bytes(c->tileT, c->K) + 31) / 32 * 32;
    a.lg_wpb = 0;
    while (pack && a.lg_wpb < 2 && (lds_wave << (a.lg_wpb + 1)) <= 65536) ++a.lg_wpb;
    const int wpb = 1 << a.lg_wpb;
    a.lds_wave = static_cast<unsigned int>(lds_wave);
    const size_t lds = lds_wave * wpb;
    const long long n_full = (c->ntiles + wpb - 1) / wpb;
    // after hop 0 the grid is sized from the longest list this forward step
    // has had, so that late, sparse forward steps do not dispatch a workgroup
    // per tile; k_hop_tail takes any tiles past the end of that grid
    long long n_tail = 0;
    // a forward step with no list seen yet borrows the longest list of the
    // nearest earlier one (else of the next one, for a hop 0 whose first list
    // covered every tile), so that a long first list still gets a full-width
    // grid rather than the narrow tail
    const int nest = static_cast<int>(c->est_tiles.size());
    long long est = hop < nest ? c->est_tiles[hop] : 0;
    for (int q = std::min(hop, nest) - 1; est == 0 && q >= 0; --q) est = c->est_tiles[q];
    if (est == 0 && hop + 1 < nest) est = c->est_tiles[hop + 1];
    const long long n_wg = hop_grid(c, hop, est, wpb, &n_tail);
    hipLaunchKernelGGL((k_hop<R, DT, S, kBar>), dim3(static_cast<unsigned>(n_wg)), dim3(64 * wpb), lds, c->stream, a);
    HIPCHK(c, hipGetLastError());
    if (hop < static_cast<int>(c->cap_tiles.size())) c->cap_tiles[hop] = n_wg < n_full ? n_wg * wpb : c->ntiles;
    if (n_tail > 0) {
        hipLaunchKernelGGL((k_hop_tail<R, DT, S, kBar>), dim3(static_cast<unsigned>(n_tail)), dim3(64 * wpb), lds,
                           c->stream, a, static_cast<unsigned int>(n_wg * wpb));
        HIPCHK(c, hipGetLastError());
    }
    return RT_OK;
}


template <typename S, bool kBar = false>
rt_status launch_hop_shape(rt_ctx* c, int hop, bool pack) {
    if (c->f32)
        return c->dl64 ? launch_hop<float, unsigned long long, S, kBar>(c, hop, pack)
                       : launch_hop<float, unsigned int, S, kBar>(c, hop, pack);
    return c->dl64 ? launch_hop<double, unsigned long long, S, kBar>(c, hop, pack)
                   : launch_hop<double, unsigned int, S, kBar>(c, hop, pack);
}

// shape: the tuned one, or (during tuning) the one this forward step times
rt_status launch_hop_any(rt_ctx* c, int hop, int shape = -1) {
    if (shape < 0) shape = c->hop_shape;
    const bool pack = shape >= kHopShapeKinds;
    const int kind = shape % kHopShapeKinds;
    // with a barrier disk or the predecessor RR scheme the forward step runs
    // the extended kernel, built in the default staging shape only (256
    // edges, 128 pairs a round): the configurations differ in packing alone
    if (c->any_bar || c->rr_orig) return launch_hop_shape<HopShape0, true>(c, hop, pack);
    if (kind == 1) return launch_hop_shape<HopShape1>(c, hop, pack);
    if (kind == 2) return launch_hop_shape<HopShape2>(c, hop, pack);
    return launch_hop_shape<HopShape0>(c, hop, pack);
}

rt_status launch_vip(rt_ctx* c, int hop) {
    VipArgs a{};
    a.hop = hop;
    a.hop0 = hop == 0;
    a.max_hops = c->p.max_hops;
    a.K = c->K;
    a.nf = c->nf;
    a.nrc = c->nrc;
    a.nec = c->nec;
    a.max_depth = c->p.max_vip_depth;
    a.dep = c->dep;
    a.seed = c->p.seed;
    a.c2 = c->c2;
    a.list = c->vip[hop & 1];
    a.vip_cap = c->vip_cap;
    a.box = c->box_d;
    a.grid = c->grid_d;
    a.cell_start = c->cell_start;
    a.cell_idx = c->cell_idx;
    a.cell_pos = c->cell_pos;
    a.pos = c->pos;
    a.xHI = c->xHI;
    a.nH = c->nH;
    a.NH = c->NH;
    a.sigma = c->sigma_d;
    a.wrc = c->rot + 9;
    a.ecd = c->ecd;
    a.rr_ecd = c->rr_ecd;
    a.xr_fx = c->xr_fx;
    a.Ufx = c->Ufx;
    a.bar = c->any_bar ? c->bar_d : nullptr;
    a.exs = c->exs;
    a.ers = c->ers;
    a.rec = c->rec;
    a.rec_next = c->rec_next;
    a.head = c->head[hop & 1];
    a.rec_cap = c->rec_cap;
    a.hot = c->hot[hop & 1];
    a.lgT = c->lgT;
    a.list_here = hop > 0 ? 1 : 0;
    a.tlist = c->tlist;
    a.rev_off = c->rev_off;
    a.N = c->N;
    a.ntiles = c->ntiles;
    a.nchunks = c->hot_len / kTileListChunk;
    a.T = c->tileT;
    a.deep = c->deep;
    a.deep_x = c->deep_x;
    a.cnt = c->cnt;
    a.act_rd = hop & 1;
    a.act_wr = (hop + 1) & 1;
    a.list_rd = hop & 1;
    a.list_wr = (hop + 1) & 1;
    a.halt_on = c->capturing ? 1 : 0;
    // workgroups for the virtual particles, after those that list the marked tiles
    const unsigned nsb = static_cast<unsigned>(std::min<long long>(1024, (c->vip_cap + 255) / 256));
    const unsigned nlist = hop > 0 ? static_cast<unsigned>(a.nchunks) : 0u;
    hipLaunchKernelGGL(k_vip_sample, dim3(nsb + nlist), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_vip_chain, dim3(1024), dim3(256), 0, c->stream, a);
    HIPCHK(c, hipGetLastError());
    // the tiles marked for this forward step: after hop 0, k_vip_sample lists
    // those the previous forward step marked and k_vip_chain appends its own;
    // hop 0's marks come from k_mark_hop0 and k_tile_list lists them (with the
    // predecessor RR scheme hop 0 runs every tile)
    if (hop == 0 && c->list0) {
        hipLaunchKernelGGL(k_mark_hop0, dim3(std::min<unsigned>(grid_for(c->ntiles, 256), 4096)), dim3(256), 0, c->stream,
                           c->rest, c->head[0], c->nrr[c->nrr_cur], c->rr_on ? 1 : 0, c->N, c->tileT, c->ntiles, c->hot[0],
                           c->cnt, c->capturing ? 1 : 0);
        HIPCHK(c, hipGetLastError());
        hipLaunchKernelGGL(k_tile_list, dim3(static_cast<unsigned>(c->hot_len / kTileListChunk)), dim3(256), 0, c->stream,
                           c->hot[0], c->ntiles, 0, -1, c->rev_off, c->N, c->tileT, c->tlist, c->cnt, c->capturing ? 1 : 0);
        HIPCHK(c, hipGetLastError());
    }
    return RT_OK;
}

__global__ void k_step_clear(const long long* cnt, int halt_on, int* head0, int* head1, long long N, double* A,
                             double* P, long long NA) {
    if (halt_on && cnt[kCntHalt] != 0) return;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < NA; t += (long long)gridDim.x * blockDim.x) {
        A[t] = 0.0;
        P[t] = 0.0;
        if (t < N) {
            head0[t] = -1;
            head1[t] = -1;
        }
    }
}

__global__ void k_set_counter(long long* cnt, int idx, long long v) {
    if (threadIdx.x == 0) cnt[idx] = v;
}

__global__ void k_clear_halt(long long* cnt) {
    if (threadIdx.x == 0) {
        cnt[kCntHalt] = 0;
        cnt[kCntDone] = 0;
    }
}

__global__ void k_step_reset(long long* cnt, long long serial, int set_serial, int halt_on) {
    if (threadIdx.x == 0 && !(halt_on && cnt[kCntHalt] != 0)) {
        if (set_serial) cnt[kCntSerial] = serial;
        cnt[kCntAct0] = 0;
        cnt[kCntAct0 + kCntLine] = 0;
        cnt[kCntVipCnt0] = 0;
        cnt[kCntVipCnt0 + 1] = 0;
        cnt[kCntRec] = 0;
        cnt[kCntHopsStep] = 0;
        cnt[kCntDone] = 0;
        cnt[kCntDeep] = 0;
        cnt[kCntTileList] = 0;
        cnt[kCntTileList + 1] = 0;
        cnt[kCntFlags] = 0;  // a step's flags are checked after it
        cnt[kCntSteps] += 1;
    }
}

__global__ void k_kappa_init(long long N, const double* xHI, const double* nH, const double* L, const int* inst_of, float* kappa) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j < N) kappa[j] = static_cast<float>(xHI[j] * nH[j] * L[inst_of[j]]);
}

rt_status fill_i32(rt_ctx* c, int* p, long long n, int v) {
    hipLaunchKernelGGL(k_fill_i32, dim3(std::min<unsigned>(grid_for(n, 256), 4096)), dim3(256), 0, c->stream, p, n, v);
    HIPCHK(c, hipGetLastError());
    return RT_OK;
}
// Exclusive scan of n ints into out[n+1]: one workgroup for short arrays,
// otherwise the three-pass scan over up to kScanBlocks workgroups.
rt_status scan_i32(rt_ctx* c, const int* in, long long n, int* out) {
    if (n <= 65536) {
        hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(1024), 0, c->stream, in, n, out);
        HIPCHK(c, hipGetLastError());
        return RT_OK;
    }
    if (!c->scan_tmp) {
        const rt_status s = alloc_n(c, &c->scan_tmp, 2ll * (kScanBlocks + 1));
        if (s != RT_OK) return s;
    }
    const long long per = (n + kScanBlocks - 1) / kScanBlocks;
    const int nb = static_cast<int>((n + per - 1) / per);
    int* sums = c->scan_tmp;
    int* offs = c->scan_tmp + kScanBlocks + 1;
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, c->stream, in, n, per, sums);
    hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(1024), 0, c->stream, sums, static_cast<long long>(nb), offs);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, c->stream, in, n, per, offs, nb, out);
    HIPCHK(c, hipGetLastError());
    return RT_OK;
}

rt_status fill_f64(rt_ctx* c, double* p, long long n, double v) {
    hipLaunchKernelGGL(k_fill_f64, dim3(std::min<unsigned>(grid_for(n, 256), 4096)), dim3(256), 0, c->stream, p, n, v);
    HIPCHK(c, hipGetLastError());
    return RT_OK;
}

#define TRY(x)                        \
    do {                              \
        rt_status s_ = (x);           \
        if (s_ != RT_OK) return s_;   \
    } while (0)

rt_status time_begin(rt_ctx* c, size_t slot) {
    if (!c->timing && !c->tuning_now) return RT_OK;
    while (c->ev.size() < 2 * (slot + 1)) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev.push_back(e);
    }
    HIPCHK(c, hipEventRecord(c->ev[2 * slot], c->stream));
    return RT_OK;
}
rt_status time_end(rt_ctx* c, size_t slot) {
    if (!c->timing && !c->tuning_now) return RT_OK;
    HIPCHK(c, hipEventRecord(c->ev[2 * slot + 1], c->stream));
    return RT_OK;
}
float elapsed(rt_ctx* c, size_t slot) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * slot], c->ev[2 * slot + 1]) != hipSuccess) return 0.f;
    return ms;
}

// Captured graphs refer to buffers, kernel variants and launch shapes: drop
// them when any of those change.
void drop_graphs(rt_ctx* c) {
    for (auto& kv : c->hop_graphs) (void)hipGraphExecDestroy(kv.second);
    c->hop_graphs.clear();
    for (auto& kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
    c->step_graphs.clear();
}

// Forward steps 1..n as one graph.  Their launches do not change from step to
// step (the step index and the stamps are read from device counters), so a
// graph is captured once per n and replayed.  If capture is not possible the
// launches are made one by one.
rt_status launch_hops_graph(rt_ctx* c, int n, bool* done) {
    *done = false;
    if (!c->graphs_ok) return RT_OK;
    auto it = c->hop_graphs.find(n);
    if (it == c->hop_graphs.end()) {
        if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            c->graphs_ok = false;
            return RT_OK;
        }
        rt_status st = RT_OK;
        for (int q = 1; q <= n && st == RT_OK; ++q) {
            st = launch_vip(c, q);
            if (st == RT_OK) st = launch_hop_any(c, q);
        }
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(c->stream, &g);
        hipGraphExec_t ex = nullptr;
        if (st != RT_OK || ec != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            c->graphs_ok = false;
            c->sticky = false;
            c->err.clear();
            return RT_OK;
        }
        (void)hipGraphDestroy(g);
        it = c->hop_graphs.emplace(n, ex).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    *done = true;
    return RT_OK;
}

// One RT step (sections 2.1 and 2.2): rotations, emission, forward steps
// until no packet is active, chemistry, ledger.
// The predecessor RR scheme's emission (before the first forward step):
// legs and cells from every emitting particle, then the arrivals per slot.
rt_status launch_rr_original(rt_ctx* c) {
    if (c->n_emit + c->N >= (1ll << 27)) return fail(c, RT_EINVAL, "predecessor RR scheme: too many emitters and particles");
    RrArgs r{};
    r.N = c->N;
    r.K = c->K;
    r.nf = c->nf;
    r.nrc = c->nrc;
    r.nec = c->nec;
    r.nsub = c->nsub;
    r.rr_bin = c->p.rr_bin;
    r.seed = c->p.seed;
    r.m0 = c->n_emit;
    r.u_ec = c->u_ec;
    r.pos = c->pos;
    r.h = c->h;
    r.ngb = c->ngb;
    r.inst_of = c->inst_of;
    r.fwd_v = c->fwd_v;
    r.f32 = c->f32 ? 1 : 0;
    r.rev_off = c->rev_off;
    r.rev_ik = c->rev_ik;
    r.nrr_prev = c->nrr[c->nrr_cur];
    r.xHI = c->xHI;
    r.nH = c->nH;
    r.sigma = c->sigma_d;
    r.wrc = c->rot + 9;
    r.bar = c->any_bar ? c->bar_d : nullptr;
    r.rr_ecd = c->rr_ecd;
    r.rr_share = c->rr_share;
    r.rr_cone = c->rr_cone;
    r.rr_pre = c->rr_pre;
    r.A = c->A;
    r.P = c->P;
    r.vip = c->vip[0];
    r.vip_cap = c->vip_cap;
    r.xr_fx = c->xr_fx;
    r.Ufx = c->Ufx;
    r.cnt = c->cnt;
    r.halt_on = c->capturing ? 1 : 0;
    hipLaunchKernelGGL(k_rr_send, dim3(grid_for(c->N * c->nsub, 64)), dim3(64), 0, c->stream, r);
    HIPCHK(c, hipGetLastError());
    const int tpb = c->nrc <= 16 ? 64 : 32;  // LDS: tpb * nrc * 48 bytes
    hipLaunchKernelGGL(k_rr_recv, dim3(grid_for(c->N, tpb)), dim3(tpb), static_cast<size_t>(tpb) * c->nrc * 48, c->stream, r);
    HIPCHK(c, hipGetLastError());
    return RT_OK;
}

// Start of an RT step: the step's accumulators cleared, the counters reset,
// rotations, emission (sources; the predecessor RR scheme), the emission
// cones' virtual particles and the first forward step.  set_serial: the stamp
// base is the host's (one step at a time); otherwise the device's own, which
// every finished step advances (steps replayed from a graph).
rt_status step_front(rt_ctx* c, bool set_serial) {
    const int ho = c->capturing ? 1 : 0;
    hipLaunchKernelGGL(k_step_clear, dim3(std::min<unsigned>(grid_for(c->N * c->nf, 256), 4096)), dim3(256), 0, c->stream,
                       c->cnt, ho, c->head[0], c->head[1], c->N, c->A, c->P, c->N * c->nf);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(64), 0, c->stream, c->cnt, c->serial, set_serial ? 1 : 0, ho);
    HIPCHK(c, hipGetLastError());
    // timing slots: 0 emission, 1 chemistry, 2 ledger, 3.. hops (vip then hop)
    TRY(time_begin(c, 0));
    StepBeginArgs sb{};
    sb.cnt = c->cnt;
    sb.halt_on = ho;
    sb.seed = c->p.seed;
    sb.nrc = c->nrc;
    sb.nec = c->nec;
    sb.nsub = c->nsub;
    sb.n_emit = c->n_emit;
    sb.u_rc = c->u_rc;
    sb.u_ec = c->u_ec;
    sb.em_kind = c->em_kind;
    sb.rot = c->rot;
    sb.wrcf = c->wrcf;
    sb.ecd = c->ecd;
    hipLaunchKernelGGL(k_step_rotations, dim3(grid_for(std::max<long long>(1, c->n_emit * c->nsub), 64)), dim3(64), 0,
                       c->stream, sb);
    HIPCHK(c, hipGetLastError());
    if (c->n_emit > 0) {
        EmitArgs ea{};
        ea.n_emit = c->n_emit;
        ea.K = c->K;
        ea.nf = c->nf;
        ea.nrc = c->nrc;
        ea.nec = c->nec;
        ea.nsub = c->nsub;
        ea.n_em = c->p.n_em;
        ea.c2 = c->c2;
        ea.em_kind = c->em_kind;
        ea.em_inst = c->em_inst;
        ea.em_pos = c->em_pos;
        ea.em_pk = c->em_pk;
        ea.em_ngb = c->em_ngb;
        ea.em_h = c->em_h;
        ea.ecd = c->ecd;
        ea.pos = c->pos;
        ea.xHI = c->xHI;
        ea.nH = c->nH;
        ea.sigma = c->sigma_d;
        ea.wrc = c->rot + 9;
        ea.rec = c->rec;
        ea.rec_next = c->rec_next;
        ea.head = c->head[0];
        ea.rec_cap = c->rec_cap;
        ea.vip = c->vip[0];
        ea.vip_cap = c->vip_cap;
        ea.cnt = c->cnt;
        ea.halt_on = ho;
        ea.xr_fx = c->xr_fx;
        ea.Ufx = c->Ufx;
        ea.bar = c->any_bar ? c->bar_d : nullptr;
        // a wavefront per (emitter, sub-step), four per workgroup
        hipLaunchKernelGGL(k_emit, dim3(grid_for(c->n_emit * c->nsub, 4)), dim3(256), 0, c->stream, ea);
        HIPCHK(c, hipGetLastError());
    }
    if (c->rr_orig) TRY(launch_rr_original(c));
    TRY(launch_vip(c, 0));
    TRY(time_end(c, 0));
    TRY(time_begin(c, 3));
    TRY(launch_hop_any(c, 0));
    TRY(time_end(c, 3));
    return RT_OK;
}

// The configuration a tuning step runs forward step q in: every
// kTuneShapes-th forward step gets the same one, and the assignment turns by
// one from one tuning step to the next, so that over the kTuneShapes tuning
// steps each configuration runs every forward-step index (their lists differ
// widely in length) about once.
int tune_shape_of(const rt_ctx* c, int q) {
    const int rot = kTuneShapes - c->tune_steps_left;
    return (q + rot) % kTuneShapes;
}

// Forward steps h, h + 1, ... one batch at a time with a host check of the
// device counters after each, until no packet is active or the cap is
// reached.  Returns the forward steps run (H) and the next unlaunched index.
rt_status hop_loop(rt_ctx* c, int h, int batch, long long* H_out, int* h_out, bool* hopcap) {
    long long H = 0;
    for (;;) {
        if (h <= c->p.max_hops) {
            const int hend = std::min(h + batch - 1, c->p.max_hops);
            if (c->p.hop_batch <= 0) batch = 1;
            bool graphed = false;
            if (!c->timing && !c->tuning_now && h == 1 && hend > 1) TRY(launch_hops_graph(c, hend, &graphed));
            for (int q = h; q <= hend && !graphed; ++q) {
                TRY(time_begin(c, 2 + 2 * q));
                TRY(launch_vip(c, q));
                TRY(time_end(c, 2 + 2 * q));
                TRY(time_begin(c, 3 + 2 * q));
                TRY(launch_hop_any(c, q, c->tuning_now ? tune_shape_of(c, q) : -1));
                TRY(time_end(c, 3 + 2 * q));
            }
            h = hend + 1;
        }
        HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->cnt, sizeof(long long) * kCntN, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        H = c->h_cnt[kCntHopsStep];
        const long long act = c->h_cnt[kCntAct0 + kCntLine * ((H + 1) & 1)];
        if (act == 0) break;
        if (H >= c->p.max_hops) {
            *hopcap = true;
            break;
        }
    }
    *H_out = H;
    *h_out = h;
    return RT_OK;
}

// End of an RT step: tallies (launched: forward-step launches of the step,
// hop 0 included), chemistry, ledger, the error check.  graph: see k_step_tally.
rt_status step_tail(rt_ctx* c, long long launched, bool graph) {
    hipLaunchKernelGGL(k_step_tally, dim3(static_cast<unsigned>(std::min<long long>(64, (c->ntiles + 255) / 256))),
                       dim3(256), 0, c->stream, c->cnt, c->part, c->ntiles, launched, graph ? 1 : 0);
    HIPCHK(c, hipGetLastError());
    // chemistry
    TRY(time_begin(c, 1));
    ChemArgs ca{};
    ca.cnt = c->cnt;
    ca.halt_on = c->capturing ? 1 : 0;
    ca.N = c->N;
    ca.nf = c->nf;
    ca.mode = c->p.recomb_mode;
    ca.isothermal = c->p.isothermal;
    ca.freeze = c->p.freeze_chem;
    ca.rr_on = c->rr_on ? 1 : 0;
    ca.dt = c->p.dt;
    ca.frac = c->p.chem_frac;
    ca.A = c->A;
    ca.dep = c->dep;
    ca.eps = c->eps_d;
    ca.nH = c->nH;
    ca.NH = c->NH;
    ca.xHI = c->xHI;
    ca.T = c->T;
    ca.nrr_wr = c->nrr[c->nrr_cur ^ 1];
    ca.kappa = c->f32 ? c->kappa : nullptr;
    ca.Linst = c->L_d;
    ca.inst_of = c->inst_of;
    ca.rc3 = c->rc3;
    hipLaunchKernelGGL(k_chem, dim3(grid_for(c->N, 256)), dim3(256), 0, c->stream, ca);
    HIPCHK(c, hipGetLastError());
    TRY(time_end(c, 1));
    // ledger
    TRY(time_begin(c, 2));
    LedgerArgs la{};
    la.cnt = c->cnt;
    la.halt_on = c->capturing ? 1 : 0;
    la.nf = c->nf;
    la.rr_bin = c->p.rr_bin;
    la.rr_on = c->rr_on ? 1 : 0;
    la.n_chunks = c->n_chunks;
    la.chunk_inst = c->chunk_inst;
    la.chunk_lo = c->chunk_lo;
    la.chunk_hi = c->chunk_hi;
    la.A = c->A;
    la.nrr_prev = c->nrr[c->nrr_cur];
    la.Fp = c->Fp;
    la.partial = c->partial;
    hipLaunchKernelGGL(k_ledger_partial, dim3(static_cast<unsigned>(c->n_chunks)), dim3(256), 0, c->stream, la);
    HIPCHK(c, hipGetLastError());
    EmitTallyArgs et{};
    et.cnt = c->cnt;
    et.halt_on = c->capturing ? 1 : 0;
    et.nf = c->nf;
    et.per_em = static_cast<long long>(c->nsub) * c->nec;
    et.em_by_inst = c->em_by_inst;
    et.em_ioff = c->em_ioff;
    et.exs = c->exs;
    et.ers = c->ers;
    et.emt = c->emt;
    hipLaunchKernelGGL(k_emit_tally, dim3(static_cast<unsigned>(c->n_inst * c->nf)), dim3(kEmTallyBlock), 0, c->stream,
                       et);
    HIPCHK(c, hipGetLastError());
    LedgerFinalArgs lf{};
    lf.n_inst = c->n_inst;
    lf.nf = c->nf;
    lf.f32 = c->f32 ? 1 : 0;
    lf.inst_chunk0 = c->inst_chunk0;
    lf.partial = c->partial;
    lf.xr_fx = c->xr_fx;
    lf.Ufx = c->Ufx;
    lf.E_src = c->E_src;
    lf.emt = c->emt;
    lf.led = c->led;
    lf.scale = c->scale;
    lf.cnt = c->cnt;
    lf.halt_on = c->capturing ? 1 : 0;
    hipLaunchKernelGGL(k_ledger_final, dim3(static_cast<unsigned>(c->n_inst * c->nf)), dim3(kLedgerFinalBlock), 0, c->stream, lf);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, c->stream, c->cnt, c->capturing ? 1 : 0);
    HIPCHK(c, hipGetLastError());
    TRY(time_end(c, 2));
    return RT_OK;
}

// The forward steps' list lengths of the last step (copied to the pinned
// mirror with the counters): the longest seen per forward step sizes its grid
// at the next launch.  Captured graphs keep the grids of their capture and
// are dropped (captured again at the next step, with grids from the new
// lengths) only when a forward step's list came within a tenth of the end of
// the grid it ran with.
void absorb_list_lengths(rt_ctx* c, long long H) {
    bool refit = false;
    const long long top = std::min<long long>(H, static_cast<long long>(c->est_tiles.size()) - 1);
    // a hop 0 that listed every tile (rest flags not known yet) says nothing
    // about the lists to come
    const long long q0 = (c->list0 && !c->rest_unknown) ? 0 : 1;
    c->rest_unknown = false;
    for (long long q = q0; q <= top; ++q) {
        const long long seen = c->h_listlen[q];
        const long long cap = c->cap_tiles[q];
        if (cap < c->ntiles && seen * 10 > cap * 9) refit = true;
        if (seen > c->est_tiles[q]) c->est_tiles[q] = seen;
    }
    if (refit) drop_graphs(c);
}

// Host bookkeeping after a step that ran H forward steps with `launched`
// launches, then the counters read back (tuning and timing use them).
rt_status step_done(rt_ctx* c, long long H, long long launched) {
    c->serial += launched;
    c->last_hops = H;
    c->nrr_cur ^= 1;
    c->step += 1;
    HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->cnt, sizeof(long long) * kCntN, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_listlen, c->listlen, sizeof(int) * c->est_tiles.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    absorb_list_lengths(c, H);
    if (c->tuning_now) {
        // forward steps whose list outgrew the main grid (the tail kernel ran
        // part of them) are left out: their time says more about the grid
        // estimate of a growing list than about the configuration
        for (long long q = 1; q <= H; ++q) {
            if (q < static_cast<long long>(c->cap_tiles.size()) && c->h_listlen[q] > c->cap_tiles[q]) continue;
            const int k = tune_shape_of(c, static_cast<int>(q));
            c->tune_ms[k] += elapsed(c, 3 + 2 * q);
            c->tune_n[k] += 1;
        }
        if (--c->tune_steps_left <= 0) {
            int best = 0;
            for (int k = 1; k < kTuneShapes; ++k)
                if (c->tune_n[k] > 0 && c->tune_ms[k] / c->tune_n[k] < c->tune_ms[best] / std::max(1ll, c->tune_n[best]))
                    best = k;
            c->hop_shape = best;
            c->tuned = true;
            drop_graphs(c);
        }
        c->tuning_now = false;
    }
    if (c->timing) {
        c->tm[4] += elapsed(c, 0);
        c->tm[3] += elapsed(c, 1);
        c->tm[5] += elapsed(c, 2);
        c->tm[0] += elapsed(c, 3);
        c->tm[1] += 1;
        for (long long q = 1; q <= H; ++q) {
            c->tm[2] += elapsed(c, 2 + 2 * q);
            c->tm[0] += elapsed(c, 3 + 2 * q);
            c->tm[1] += 1;
        }
    }
    return RT_OK;
}

// Stamps are 30-bit: restart them (and forget every old mark) long before they wrap.
rt_status restart_stamps_if_needed(rt_ctx* c, long long ahead) {
    if (c->serial + ahead + c->p.max_hops + 2 < (1ll << 30)) return RT_OK;
    for (int b = 0; b < 2; ++b) {
        HIPCHK(c, hipMemsetAsync(c->inbox[b], 0xff, c->inbox_bytes, c->stream));
        TRY(fill_i32(c, c->hot[b], c->hot_len, -1));
    }
    c->serial = 0;
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, c->stream, c->cnt, static_cast<int>(kCntSerial), 0ll);
    HIPCHK(c, hipGetLastError());
    return RT_OK;
}

// One RT step, checked by the host as it goes (used while tuning or timing,
// before the forward-step count of a step is known, and with a fixed batch).
rt_status one_step(rt_ctx* c, bool* hopcap) {
    // The autotuner times the forward-step shapes on steps whose work is
    // representative (at least 16 forward steps in the previous step),
    // alternating the shape from one forward step to the next.
    c->tuning_now = c->tune_mode < 0 && !c->tuned && (c->last_hops >= 16 || c->tune_mode == -2);
    TRY(restart_stamps_if_needed(c, 0));
    TRY(step_front(c, true));
    // Forward steps are enqueued in batches between host checks of the device
    // counters.  Automatic batching enqueues one more than the previous step
    // needed (a step rarely needs more than one extra: launches past the end
    // exit at once, cheaper than a host round trip), then goes one at a time.
    const int batch = c->p.hop_batch > 0 ? c->p.hop_batch : std::max(1, static_cast<int>(c->last_hops) + 1);
    long long H = 0;
    int h = 1;
    TRY(hop_loop(c, 1, batch, &H, &h, hopcap));
    TRY(step_tail(c, h, false));
    return step_done(c, H, h);
}

// The whole RT step with hg forward steps after hop 0, captured once per
// (hg, parity of the RR double buffer) and replayed: no host check inside.
rt_status step_graph(rt_ctx* c, int hg, hipGraphExec_t* out) {
    const long long key = 2ll * hg + c->nrr_cur;
    auto it = c->step_graphs.find(key);
    if (it != c->step_graphs.end()) {
        *out = it->second;
        return RT_OK;
    }
    *out = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        c->graphs_ok = false;
        return RT_OK;
    }
    c->capturing = true;
    rt_status st = step_front(c, false);
    for (int q = 1; q <= hg && st == RT_OK; ++q) {
        st = launch_vip(c, q);
        if (st == RT_OK) st = launch_hop_any(c, q);
    }
    if (st == RT_OK) st = step_tail(c, hg + 1, true);
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->stream, &g);
    hipGraphExec_t ex = nullptr;
    if (st != RT_OK || ec != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->graphs_ok = false;
        c->sticky = false;
        c->err.clear();
        return RT_OK;
    }
    (void)hipGraphDestroy(g);
    c->step_graphs.emplace(key, ex);
    *out = ex;
    return RT_OK;
}

// Up to n RT steps, each replayed from its whole-step graph and enqueued
// back to back with a single host check at the end.  A step that needs more
// forward steps than its graph holds halts the queue on the device; it is
// finished here one forward step at a time.  Returns the steps finished.
rt_status graph_steps(rt_ctx* c, int n, int* done, bool* hopcap) {
    *done = 0;
    // forward steps a step graph holds: at least two more than the last step
    // needed, rounded up to a multiple of four, so that a step whose fronts
    // grew rarely halts the queue and one graph serves several steps (an idle
    // forward step costs its four launches, ~15 us; a halt a host round trip
    // per forward step and often a new capture)
    const int hg = static_cast<int>(std::min<long long>(c->p.max_hops, (c->last_hops + 2 + 3) / 4 * 4));
    TRY(restart_stamps_if_needed(c, static_cast<long long>(hg + 1) * n));
    const long long step0 = c->step;
    const int cur0 = c->nrr_cur;
    int launched_steps = 0;
    for (int s = 0; s < n; ++s) {
        hipGraphExec_t ex = nullptr;
        TRY(step_graph(c, hg, &ex));
        if (!ex) break;  // capture not possible: the caller goes on step by step
        HIPCHK(c, hipGraphLaunch(ex, c->stream));
        c->nrr_cur ^= 1;
        ++launched_steps;
    }
    HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->cnt, sizeof(long long) * kCntN, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_listlen, c->listlen, sizeof(int) * c->est_tiles.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long halt = c->h_cnt[kCntHalt];
    const long long started = c->h_cnt[kCntSteps] - step0;  // the step counter counts a step at its start
    const long long finished = halt == 1 ? started - 1 : started;
    c->step = step0 + finished;
    c->nrr_cur = cur0 ^ static_cast<int>(finished & 1);
    c->serial = c->h_cnt[kCntSerial];
    if (finished > 0) c->last_hops = c->h_cnt[kCntLastHops];
    if (finished > 0) absorb_list_lengths(c, c->last_hops);
    *done = static_cast<int>(finished);
    if (halt == 0) return RT_OK;
    hipLaunchKernelGGL(k_clear_halt, dim3(1), dim3(64), 0, c->stream, c->cnt);
    HIPCHK(c, hipGetLastError());
    if (halt == 2) return RT_OK;  // the error flags of the last finished step are reported by the caller
    // finish the halted step: its first hg forward steps ran
    long long H = 0;
    int h = hg + 1;
    TRY(hop_loop(c, hg + 1, 1, &H, &h, hopcap));
    TRY(step_tail(c, h, false));
    TRY(step_done(c, H, h));
    *done += 1;
    return RT_OK;
}

// Input arrays may be host or device memory: device (and managed) arrays are
// copied to the host first, since validation and set-up read them there.
// Returns p itself for host memory, nullptr if the copy failed.
template <typename T>
const T* staged(const T* p, size_t n, std::vector<T>& buf) {
    if (!p || n == 0) return p;
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable host memory is unknown to the runtime
        return p;
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) return p;
    buf.resize(n);
    if (hipMemcpy(buf.data(), p, n * sizeof(T), hipMemcpyDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return buf.data();
}

}  // namespace

extern "C" {

const char* rt_last_error(const rt_ctx* c) { return c ? c->err.c_str() : "null context"; }

namespace {
rt_status init_impl(rt_ctx** out, const rt_params* p, const double* sigma_nu, const double* eps_nu, int32_t n_inst,
                    const int64_t* inst_off, const double* box, const double* pos, const double* n_H, const double* N_H,
                    const double* x_HI0, const double* T0, void* hip_stream);
}  // namespace

rt_status rt_init(rt_ctx** out, const rt_params* p, const double* sigma_nu, const double* eps_nu, int32_t n_inst,
                  const int64_t* inst_off, const double* box, const double* pos, const double* n_H, const double* N_H,
                  const double* x_HI0, const double* T0, void* hip_stream) {
    if (!out || !p || !sigma_nu || !eps_nu || !inst_off || !box || !pos || !n_H || !N_H || !x_HI0 || !T0 || n_inst < 1 ||
        p->n_freq < 1 || p->n_freq > 15)
        return RT_EINVAL;
    std::vector<int64_t> off_h;
    const int64_t* off = staged(inst_off, static_cast<size_t>(n_inst) + 1, off_h);
    if (!off) return RT_EINVAL;
    const long long N = off[n_inst];
    if (off[0] != 0 || N <= 0 || N >= (1ll << 26)) return RT_EINVAL;
    std::vector<double> sg, ep, bx, ps, nh, NHh, xh, th;
    const double* a0 = staged(sigma_nu, p->n_freq, sg);
    const double* a1 = staged(eps_nu, p->n_freq, ep);
    const double* a2 = staged(box, 6 * static_cast<size_t>(n_inst), bx);
    const double* a3 = staged(pos, 3 * static_cast<size_t>(N), ps);
    const double* a4 = staged(n_H, N, nh);
    const double* a5 = staged(N_H, N, NHh);
    const double* a6 = staged(x_HI0, N, xh);
    const double* a7 = staged(T0, N, th);
    if (!a0 || !a1 || !a2 || !a3 || !a4 || !a5 || !a6 || !a7) return RT_EINVAL;
    return init_impl(out, p, a0, a1, n_inst, off, a2, a3, a4, a5, a6, a7, hip_stream);
}

namespace {
rt_status init_impl(rt_ctx** out, const rt_params* p, const double* sigma_nu, const double* eps_nu, int32_t n_inst,
                    const int64_t* inst_off, const double* box, const double* pos, const double* n_H, const double* N_H,
                    const double* x_HI0, const double* T0, void* hip_stream) {
    if (!out || !p || !sigma_nu || !eps_nu || !inst_off || !box || !pos || !n_H || !N_H || !x_HI0 || !T0)
        return RT_EINVAL;
    *out = nullptr;
    if (p->n_ngb < 1 || p->n_ngb > kMaxNgb || p->n_tc < 3 || !pow2(p->n_rc) || p->n_rc > 32 || p->n_ec < 1 ||
        p->n_ec > 64 || p->n_freq < 1 || p->n_freq > 15 || p->rr_bin >= p->n_freq || p->rr_bin < -1 ||
        p->recomb_mode < 0 || p->recomb_mode > 3 ||
        ((p->recomb_mode == RT_RR_TRANSPORT || p->recomb_mode == RT_RR_ORIGINAL) && p->rr_bin < 0) ||
        p->precision < 0 || p->precision > 1 || p->n_em < 1 || p->n_em > 4095 || p->max_hops < 0 ||
        p->max_hops > 4095 || p->max_vip_depth < 1 || p->max_vip_depth > 15 || !(p->dt > 0.0) ||
        !(p->floor_rel >= 0.0) || !(p->chem_frac > 0.0) || n_inst < 1)
        return RT_EINVAL;
    if (inst_off[0] != 0) return RT_EINVAL;
    for (int k = 0; k < n_inst; ++k) {
        if (inst_off[k + 1] - inst_off[k] <= p->n_ngb) return RT_EINVAL;
        for (int a = 0; a < 3; ++a)
            if (!(box[6 * k + 3 + a] > box[6 * k + a])) return RT_EINVAL;
        for (long long i = inst_off[k]; i < inst_off[k + 1]; ++i) {
            for (int a = 0; a < 3; ++a)
                if (!(pos[3 * i + a] >= box[6 * k + a] && pos[3 * i + a] <= box[6 * k + 3 + a])) return RT_EINVAL;
            if (!(n_H[i] > 0.0) || !(N_H[i] > 0.0) || !(x_HI0[i] >= 0.0 && x_HI0[i] <= 1.0) || !(T0[i] > 0.0))
                return RT_EINVAL;
        }
    }
    const long long N = inst_off[n_inst];
    // particle indices are packed into 26 bits of the edge lists; the slots of
    // one particle (N_RC x N_freq) form an aligned power-of-two lane group
    if (N >= (1ll << 26) || N * static_cast<long long>(p->n_ngb) >= (1ll << 31) - 1) return RT_EINVAL;
    if (!pow2(p->n_rc * p->n_freq) || p->n_rc * p->n_freq > 64) return RT_EINVAL;
    rt_ctx* c = new rt_ctx();
    c->p = *p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->dev) != hipSuccess) {
        delete c;
        return RT_EDEVICE;
    }
    c->N = N;
    c->n_inst = n_inst;
    c->nf = p->n_freq;
    c->nrc = p->n_rc;
    c->nec = p->n_ec;
    c->G = p->n_rc * p->n_freq;
    c->K = p->n_ngb;
    c->B = N * c->G;
    c->f32 = p->precision == RT_FP32;
    c->dl64 = c->G > 32;
    {
        // a tile is one wavefront; its LDS (at most 24 KiB) bounds the particles per tile
        auto hop_lds = [&](int t) {
            if (c->f32)
                return c->dl64 ? HopLds<float, unsigned long long>::bytes(t, c->K) : HopLds<float, unsigned int>::bytes(t, c->K);
            return c->dl64 ? HopLds<double, unsigned long long>::bytes(t, c->K) : HopLds<double, unsigned int>::bytes(t, c->K);
        };
        int T = 64 / c->G;
        while (T > 1 && hop_lds(T) > 24 * 1024) T /= 2;
        c->tileT = T;
        while ((1 << c->lgT) < T) ++c->lgT;
    }
    c->rr_on = p->recomb_mode == RT_RR_TRANSPORT || p->recomb_mode == RT_RR_ORIGINAL;
    c->rr_orig = p->recomb_mode == RT_RR_ORIGINAL;
    // the predecessor scheme's arrivals are summed per slot for hop 0, which
    // then runs every tile
    c->list0 = !c->rr_orig;
    const double cc = 1.0 - 2.0 / static_cast<double>(p->n_tc);
    c->c2 = cc * cc;
    c->inst_off.assign(inst_off, inst_off + n_inst + 1);
    c->box.assign(box, box + 6 * n_inst);
    c->sigma.assign(sigma_nu, sigma_nu + c->nf);
    c->eps.assign(eps_nu, eps_nu + c->nf);
    c->nsub = p->n_em;
    auto bail = [&](rt_status s) {
        rt_destroy(c);
        return s;
    };
#define ITRY(x)                      \
    do {                             \
        rt_status s_ = (x);          \
        if (s_ != RT_OK) return bail(s_); \
    } while (0)
    // per-instance constants: box side, photon unit (mean N_H, for FP32 bins), clock factor
    std::vector<int> inst_of(N);
    c->U.assign(n_inst, 1.0);
    c->L.assign(n_inst, 1.0);
    std::vector<float> clf(n_inst);
    std::vector<double> mean_NH(n_inst);
    std::vector<GridInfo> grid(n_inst);
    long long ncell = 0;
    for (int k = 0; k < n_inst; ++k) {
        const long long n = inst_off[k + 1] - inst_off[k];
        double sum = 0.0;
        for (long long i = inst_off[k]; i < inst_off[k + 1]; ++i) {
            inst_of[i] = k;
            sum += N_H[i];
        }
        double Lmax = 0.0, vol = 1.0;
        GridInfo& g = grid[k];
        for (int a = 0; a < 3; ++a) {
            const double La = box[6 * k + 3 + a] - box[6 * k + a];
            Lmax = std::max(Lmax, La);
            vol *= La;
        }
        c->U[k] = c->f32 ? sum / static_cast<double>(n) : 1.0;
        mean_NH[k] = sum / static_cast<double>(n);
        c->L[k] = Lmax;
        clf[k] = static_cast<float>(Lmax / (kCLight * p->dt));
        // cells of ~2 particles on average; where the particles cluster (the
        // fullest cell holds more than kCellDense), finer until the fullest
        // would hold about kCellDense (at most 8x per axis and 1024 cells per
        // axis), so that neighbour searches in dense regions sort fewer
        // candidates (the search is exact whatever the cells)
        double cs = std::cbrt(2.0 * vol / static_cast<double>(n));
        auto set_cells = [&](double csz) {
            for (int a = 0; a < 3; ++a) {
                const double La = box[6 * k + 3 + a] - box[6 * k + a];
                int m = static_cast<int>(La / csz);
                m = std::max(1, std::min(m, 1024));
                g.nc[a] = m;
                g.cs[a] = La / m;
                g.lo[a] = box[6 * k + a];
            }
        };
        set_cells(cs);
        {
            std::vector<int> occ(static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2], 0);
            int most = 0;
            for (long long i = inst_off[k]; i < inst_off[k + 1]; ++i) {
                int ci[3];
                for (int a = 0; a < 3; ++a)
                    ci[a] = std::max(0, std::min(g.nc[a] - 1, static_cast<int>((pos[3 * i + a] - g.lo[a]) / g.cs[a])));
                most = std::max(most, ++occ[(static_cast<size_t>(ci[0]) * g.nc[1] + ci[1]) * g.nc[2] + ci[2]]);
            }
            if (most > kCellDense) set_cells(cs / std::min(8.0, std::cbrt(static_cast<double>(most) / kCellDense)));
        }
        g.cell0 = ncell;
        ncell += static_cast<long long>(g.nc[0]) * g.nc[1] * g.nc[2];
    }
    // FP32 positions in units of the instance's box side, relative to its corner
    std::vector<double> floor_d(N);
    std::vector<float> floor_f(c->f32 ? N : 1);
    for (long long i = 0; i < N; ++i) {
        floor_d[i] = p->floor_rel * N_H[i];
        if (c->f32) floor_f[i] = static_cast<float>(floor_d[i] / c->U[inst_of[i]]);
    }
    std::vector<float> sigf(c->nf);
    for (int nu = 0; nu < c->nf; ++nu) sigf[nu] = static_cast<float>(c->sigma[nu]);
    std::vector<double> urc, uec;
    direction_set(c->nrc, urc);
    direction_set(c->nec, uec);

    ITRY(upload(c, &c->inst_of, inst_of.data(), N));
    ITRY(upload(c, &c->box_d, box, 6ll * n_inst));
    ITRY(upload(c, &c->pos, pos, 3 * N));
    ITRY(upload(c, &c->nH, n_H, N));
    ITRY(upload(c, &c->NH, N_H, N));
    ITRY(upload(c, &c->xHI, x_HI0, N));
    ITRY(upload(c, &c->T, T0, N));
    if (p->isothermal || p->freeze_chem) {  // temperatures never change: rates evaluated once
        ITRY(alloc_n(c, &c->rc3, 3 * N));
        hipLaunchKernelGGL(k_rates_cache, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->T, c->rc3);
        HIPCHK(c, hipGetLastError());
    }
    ITRY(upload(c, &c->sigma_d, c->sigma.data(), c->nf));
    ITRY(upload(c, &c->sigmaf_d, sigf.data(), c->nf));
    ITRY(upload(c, &c->eps_d, c->eps.data(), c->nf));
    ITRY(upload(c, &c->U_d, c->U.data(), n_inst));
    ITRY(upload(c, &c->L_d, c->L.data(), n_inst));
    ITRY(upload(c, &c->clf_d, clf.data(), n_inst));
    ITRY(upload(c, &c->u_rc, urc.data(), 3ll * c->nrc));
    ITRY(upload(c, &c->u_ec, uec.data(), 3ll * c->nec));
    ITRY(upload(c, &c->grid_d, grid.data(), n_inst));
    if (c->f32) {
        float* fb = nullptr;
        ITRY(upload(c, &fb, floor_f.data(), N));
        c->floor_b = fb;
        ITRY(alloc_n(c, &c->kappa, N));
    } else {
        double* fb = nullptr;
        ITRY(upload(c, &fb, floor_d.data(), N));
        c->floor_b = fb;
    }
    ITRY(alloc_n(c, &c->h, N));
    ITRY(alloc_n(c, &c->ngb, N * c->K));
    ITRY(alloc_n(c, &c->rot, 9 + 3ll * c->nrc));
    ITRY(alloc_n(c, &c->wrcf, 3ll * c->nrc));
    // neighbour search: counting sort into cells, then exact kNN per particle
    int *cell_of = nullptr, *cnt = nullptr, *cursor = nullptr;
    ITRY(alloc_n(c, &cell_of, N));
    ITRY(alloc_n(c, &cnt, ncell));
    ITRY(alloc_n(c, &cursor, std::max<long long>(ncell, N)));
    ITRY(alloc_n(c, &c->cell_start, ncell + 1));
    ITRY(alloc_n(c, &c->cell_idx, N));
    ITRY(fill_i32(c, cnt, ncell, 0));
    ITRY(fill_i32(c, cursor, std::max<long long>(ncell, N), 0));
    hipLaunchKernelGGL(k_cell_count, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->pos, c->inst_of, c->grid_d,
                       cell_of, cnt);
    ITRY(scan_i32(c, cnt, ncell, c->cell_start));
    hipLaunchKernelGGL(k_cell_fill, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, cell_of, c->cell_start, cursor,
                       c->cell_idx);
    ITRY(alloc_n(c, &c->cell_pos, 3 * N));
    hipLaunchKernelGGL(k_cell_pos, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->cell_idx, c->pos, c->cell_pos);
    hipLaunchKernelGGL(k_knn_wave, dim3(static_cast<unsigned>(std::min<long long>((N + 3) / 4, 8192))), dim3(256), 0,
                       c->stream, N, c->pos, c->inst_of, c->grid_d, c->cell_start, c->cell_idx, c->cell_pos, c->K,
                       c->ngb, c->h);
    // reverse lists, sorted by sender
    ITRY(alloc_n(c, &c->rev_off, N + 1));
    ITRY(alloc_n(c, &c->rev_src, N * c->K));
    ITRY(alloc_n(c, &c->rev_pos, N * c->K));
    int* rcnt = nullptr;
    ITRY(alloc_n(c, &rcnt, N));
    ITRY(fill_i32(c, rcnt, N, 0));
    ITRY(fill_i32(c, cursor, N, 0));
    hipLaunchKernelGGL(k_rev_count, dim3(grid_for(N * c->K, 256)), dim3(256), 0, c->stream, N * c->K, c->ngb, rcnt);
    ITRY(scan_i32(c, rcnt, N, c->rev_off));
    hipLaunchKernelGGL(k_rev_fill, dim3(grid_for(N * c->K, 256)), dim3(256), 0, c->stream, N, c->K, c->ngb, c->rev_off,
                       cursor, c->rev_src, c->rev_pos);
    hipLaunchKernelGGL(k_rev_sort, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->rev_off, c->rev_src,
                       c->rev_pos);
    HIPCHK(c, hipGetLastError());
    // packed reverse edges and the offsets the forward step needs
    ITRY(alloc_n(c, &c->rev_ik, N * c->K));
    ITRY(dalloc(c, &c->rev_v, (c->f32 ? 16 : 32) * static_cast<size_t>(N * c->K)));
    ITRY(dalloc(c, &c->fwd_v, (c->f32 ? 16 : 32) * static_cast<size_t>(N * c->K)));
    if (c->f32)
        hipLaunchKernelGGL(k_edge_vectors<float4>, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->K, c->pos,
                           c->ngb, c->rev_off, c->rev_src, c->rev_pos, c->inst_of, c->L_d, c->rev_ik,
                           static_cast<float4*>(c->rev_v), static_cast<float4*>(c->fwd_v));
    else
        hipLaunchKernelGGL(k_edge_vectors<double4>, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->K, c->pos,
                           c->ngb, c->rev_off, c->rev_src, c->rev_pos, c->inst_of, c->L_d, c->rev_ik,
                           static_cast<double4*>(c->rev_v), static_cast<double4*>(c->fwd_v));
    HIPCHK(c, hipGetLastError());
    // bins and work buffers
    const size_t rsz = c->f32 ? sizeof(float) : sizeof(double);
    c->ntiles = (N + c->tileT - 1) / c->tileT;
    ITRY(dalloc(c, &c->pk, 4 * rsz * c->B));
    ITRY(dalloc(c, &c->pcl, rsz * c->B));
    ITRY(alloc_n(c, &c->cm, c->B));
    HIPCHK(c, hipMemsetAsync(c->pk, 0, 4 * rsz * c->B, c->stream));
    HIPCHK(c, hipMemsetAsync(c->pcl, 0, rsz * c->B, c->stream));
    HIPCHK(c, hipMemsetAsync(c->cm, 0, 8 * c->B, c->stream));
    for (int b = 0; b < 2; ++b) {
        ITRY(dalloc(c, &c->mv[b], 4 * rsz * c->B));
        ITRY(dalloc(c, &c->mvc[b], 2 * rsz * c->B));
        // inbox tags start all-ones: no stamp matches
        c->inbox_bytes = (c->dl64 ? sizeof(Inbox<unsigned long long>) : sizeof(Inbox<unsigned int>)) *
                         static_cast<size_t>(N * c->K);
        ITRY(dalloc(c, &c->inbox[b], c->inbox_bytes));
        HIPCHK(c, hipMemsetAsync(c->inbox[b], 0xff, c->inbox_bytes, c->stream));
        c->hot_len = (c->ntiles + kTileListChunk - 1) / kTileListChunk * kTileListChunk;
        ITRY(alloc_n(c, &c->hot[b], c->hot_len));
        ITRY(fill_i32(c, c->hot[b], c->hot_len, -1));
        if (b == 0) {
            ITRY(alloc_n(c, &c->part, 3 * c->ntiles));
            ITRY(alloc_n(c, &c->tlist, c->ntiles));
            HIPCHK(c, hipMemsetAsync(c->part, 0, sizeof(unsigned long long) * 3 * c->ntiles, c->stream));
            // until a tile has run, whether photons rest in it is not known:
            // every tile runs at the first hop 0
            ITRY(alloc_n(c, &c->rest, c->ntiles));
            ITRY(fill_i32(c, c->rest, c->ntiles, 1));
        }
        ITRY(alloc_n(c, &c->nrr[b], N));
        ITRY(fill_f64(c, c->nrr[b], N, 0.0));
        ITRY(alloc_n(c, &c->head[b], N));
    }
    if (c->rr_orig) {
        ITRY(alloc_n(c, &c->rr_ecd, 3ll * N * c->nsub * c->nec));
        ITRY(alloc_n(c, &c->rr_share, N * c->K * static_cast<long long>(c->nsub)));
        ITRY(alloc_n(c, &c->rr_cone, N * c->K * static_cast<long long>(c->nsub)));
        ITRY(alloc_n(c, &c->rr_pre, 6ll * N * c->nrc));
    }
    ITRY(alloc_n(c, &c->A, N * c->nf));
    ITRY(alloc_n(c, &c->P, N * c->nf));
    ITRY(fill_f64(c, c->A, N * c->nf, 0.0));
    ITRY(alloc_n(c, &c->dep, 3 * N * c->nf));
    HIPCHK(c, hipMemsetAsync(c->dep, 0, sizeof(long long) * 3 * N * c->nf, c->stream));
    ITRY(fill_f64(c, c->P, N * c->nf, 0.0));
    ITRY(alloc_n(c, &c->Fp, N * c->nf));
    ITRY(fill_f64(c, c->Fp, N * c->nf, 0.0));
    ITRY(alloc_n(c, &c->xr_fx, 6ll * n_inst * c->nf));
    HIPCHK(c, hipMemsetAsync(c->xr_fx, 0, sizeof(unsigned long long) * 6 * n_inst * c->nf, c->stream));
    ITRY(upload(c, &c->Ufx, mean_NH.data(), n_inst));
    c->bar.assign(4 * static_cast<size_t>(n_inst), 0.0);
    ITRY(upload(c, &c->bar_d, c->bar.data(), 4ll * n_inst));
    // default: room for every slot whose transmission cone is empty, the
    // chance of which is (1 - 1/N_TC)^N_ngb for neighbours spread evenly over
    // directions (a cone covers 1/N_TC of the sphere): ~5% at N_TC = 16,
    // ~70% at N_TC = 128 with 48 neighbours
    const double f_empty = std::pow(1.0 - 1.0 / p->n_tc, static_cast<double>(p->n_ngb));
    c->vip_cap = p->vip_capacity > 0 ? p->vip_capacity
                                     : std::max({1ll << 16, c->B / 8, static_cast<long long>(std::ceil(c->B * f_empty))});
    c->rec_cap = p->record_capacity > 0 ? p->record_capacity : std::max<long long>(1 << 20, c->vip_cap * 4);
    if (c->rec_cap >= (1ll << 31)) c->rec_cap = (1ll << 31) - 1;
    for (int b = 0; b < 2; ++b) ITRY(alloc_n(c, &c->vip[b], c->vip_cap));
    ITRY(alloc_n(c, &c->deep, c->vip_cap));
    ITRY(alloc_n(c, &c->deep_x, 3 * c->vip_cap));
    ITRY(alloc_n(c, &c->rec, c->rec_cap));
    ITRY(alloc_n(c, &c->rec_next, c->rec_cap));
    ITRY(alloc_n(c, &c->cnt, kCntN));
    HIPCHK(c, hipMemsetAsync(c->cnt, 0, sizeof(long long) * kCntN, c->stream));
    HIPCHK(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_cnt), sizeof(long long) * kCntN, hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_listlen), sizeof(int) * (p->max_hops + 2), hipHostMallocDefault));
    ITRY(alloc_n(c, &c->listlen, p->max_hops + 2ll));
    ITRY(fill_i32(c, c->listlen, p->max_hops + 2ll, 0));
    c->est_tiles.assign(p->max_hops + 2, 0);
    c->cap_tiles.assign(p->max_hops + 2, 0);
    ITRY(alloc_n(c, &c->led, 5ll * n_inst * c->nf));
    ITRY(fill_f64(c, c->led, 5ll * n_inst * c->nf, 0.0));
    ITRY(alloc_n(c, &c->scale, 1ll * n_inst * c->nf));
    ITRY(fill_f64(c, c->scale, 1ll * n_inst * c->nf, 1.0));
    // ledger chunks: fixed ranges of particles inside one instance
    std::vector<int> ci;
    std::vector<long long> clo, chi, c0(n_inst + 1, 0);
    for (int k = 0; k < n_inst; ++k) {
        c0[k] = static_cast<long long>(ci.size());
        for (long long a = inst_off[k]; a < inst_off[k + 1]; a += kChunk) {
            ci.push_back(k);
            clo.push_back(a);
            chi.push_back(std::min<long long>(a + kChunk, inst_off[k + 1]));
        }
    }
    c0[n_inst] = static_cast<long long>(ci.size());
    c->n_chunks = static_cast<long long>(ci.size());
    ITRY(upload(c, &c->chunk_inst, ci.data(), c->n_chunks));
    ITRY(upload(c, &c->chunk_lo, clo.data(), c->n_chunks));
    ITRY(upload(c, &c->chunk_hi, chi.data(), c->n_chunks));
    ITRY(upload(c, &c->inst_chunk0, c0.data(), n_inst + 1));
    ITRY(alloc_n(c, &c->partial, c->n_chunks * c->nf * 3));
    if (c->f32) {
        hipLaunchKernelGGL(k_kappa_init, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, c->xHI, c->nH, c->L_d,
                           c->inst_of, c->kappa);
        HIPCHK(c, hipGetLastError());
    }
    // no sources yet
    c->n_emit = 0;
    ITRY(alloc_n(c, &c->E_src, 1ll * n_inst * c->nf));
    ITRY(fill_f64(c, c->E_src, 1ll * n_inst * c->nf, 0.0));
    ITRY(alloc_n(c, &c->em_inst, 1));
    ITRY(alloc_n(c, &c->em_kind, 1));
    ITRY(alloc_n(c, &c->ecd, 3));
    ITRY(alloc_n(c, &c->exs, 1));
    ITRY(alloc_n(c, &c->ers, 1));
    ITRY(alloc_n(c, &c->em_by_inst, 1));
    {
        const std::vector<long long> zero(n_inst + 1, 0);
        ITRY(upload(c, &c->em_ioff, zero.data(), n_inst + 1ll));
    }
    ITRY(alloc_n(c, &c->emt, 2ll * n_inst * c->nf));
    ITRY(resolve_scratch(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
#undef ITRY
    *out = c;
    return RT_OK;
}
}  // namespace

namespace {
rt_status add_sources_impl(rt_ctx* c, int32_t n_src, const int32_t* inst, const int32_t* kind, const double* pos,
                           const double* rate, const int32_t* n_side);
}  // namespace

rt_status rt_add_sources(rt_ctx* c, int32_t n_src, const int32_t* inst, const int32_t* kind, const double* pos,
                         const double* rate, const int32_t* n_side) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    if (n_src < 0) return fail(c, RT_EINVAL, "n_src < 0");
    std::vector<int32_t> ih, kh, nh;
    std::vector<double> ph, rh;
    const int32_t* i1 = staged(inst, n_src, ih);
    const int32_t* k1 = staged(kind, n_src, kh);
    const double* p1 = staged(pos, 3 * static_cast<size_t>(n_src), ph);
    const double* r1 = staged(rate, static_cast<size_t>(n_src) * c->nf, rh);
    const int32_t* n1 = staged(n_side, n_src, nh);
    if ((inst && !i1) || (kind && !k1) || (pos && !p1) || (rate && !r1) || (n_side && !n1))
        return fail(c, RT_EINVAL, "source arrays could not be read");
    return add_sources_impl(c, n_src, i1, k1, p1, r1, n1);
}

namespace {
rt_status add_sources_impl(rt_ctx* c, int32_t n_src, const int32_t* inst, const int32_t* kind, const double* pos,
                           const double* rate, const int32_t* n_side) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    if (n_src < 0 || (n_src > 0 && (!inst || !kind || !pos || !rate))) return fail(c, RT_EINVAL, "null source arrays");
    long long total = 0;
    for (int s = 0; s < n_src; ++s) {
        if (inst[s] < 0 || inst[s] >= c->n_inst) return fail(c, RT_EINVAL, "source instance out of range");
        if (kind[s] == RT_SRC_POINT) {
            const double* bx = &c->box[6 * inst[s]];
            for (int a = 0; a < 3; ++a)
                if (!(pos[3 * s + a] >= bx[a] && pos[3 * s + a] <= bx[3 + a]))
                    return fail(c, RT_EINVAL, "point source outside its box");
            total += 1;
        } else if (kind[s] == RT_SRC_PLANE_XLO) {
            if (!n_side || n_side[s] < 1 || n_side[s] > 4096) return fail(c, RT_EINVAL, "bad plane n_side");
            total += static_cast<long long>(n_side[s]) * n_side[s];
        } else {
            return fail(c, RT_EINVAL, "bad source kind");
        }
        for (int nu = 0; nu < c->nf; ++nu)
            if (!(rate[s * c->nf + nu] >= 0.0) || !std::isfinite(rate[s * c->nf + nu]))
                return fail(c, RT_EINVAL, "bad source rate");
    }
    if (total >= (1ll << 24)) return fail(c, RT_EINVAL, "too many emitters");
    std::vector<int> ek(total), ei(total);
    std::vector<double> ep(3 * total), epk(total * c->nf);
    std::vector<double> esrc(static_cast<size_t>(c->n_inst) * c->nf, 0.0);
    long long m = 0;
    const double dt = c->p.dt;
    for (int s = 0; s < n_src; ++s) {
        const int k = inst[s];
        const double* bx = &c->box[6 * k];
        if (kind[s] == RT_SRC_POINT) {
            ek[m] = 0;
            ei[m] = k;
            for (int a = 0; a < 3; ++a) ep[3 * m + a] = pos[3 * s + a];
            for (int nu = 0; nu < c->nf; ++nu) {
                const double pk = rate[s * c->nf + nu] * dt / static_cast<double>(c->p.n_em * c->p.n_ec);
                epk[m * c->nf + nu] = pk;
                if (pk > 0.0) esrc[k * c->nf + nu] += pk * c->p.n_em * c->p.n_ec;
            }
            ++m;
        } else {
            const int n = n_side[s];
            const double dy = (bx[4] - bx[1]) / n, dz = (bx[5] - bx[2]) / n;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    ek[m] = 1;
                    ei[m] = k;
                    ep[3 * m] = bx[0];
                    ep[3 * m + 1] = bx[1] + (static_cast<double>(a) + 0.5) * dy;
                    ep[3 * m + 2] = bx[2] + (static_cast<double>(b) + 0.5) * dz;
                    for (int nu = 0; nu < c->nf; ++nu) {
                        const double pk = rate[s * c->nf + nu] * dt * (dy * dz);
                        epk[m * c->nf + nu] = pk;
                        if (pk > 0.0) esrc[k * c->nf + nu] += pk;
                    }
                    ++m;
                }
        }
    }
    // emitters grouped by instance, in emitter order within each (counting sort)
    std::vector<long long> ioff(c->n_inst + 1, 0);
    for (long long q = 0; q < total; ++q) ioff[ei[q] + 1] += 1;
    for (int k = 0; k < c->n_inst; ++k) ioff[k + 1] += ioff[k];
    std::vector<long long> cur(ioff.begin(), ioff.end() - 1);
    std::vector<int> by_inst(total);
    for (long long q = 0; q < total; ++q) by_inst[cur[ei[q]]++] = static_cast<int>(q);
    // The new buffers are built first: if one cannot be allocated, they are
    // freed again and the context keeps its sources.
    const long long necd = std::max<long long>(1, total * c->nsub * c->nec);
    int *n_kind = nullptr, *n_inst = nullptr, *n_ngb = nullptr, *n_by = nullptr;
    double *n_pos = nullptr, *n_pk = nullptr, *n_E = nullptr, *n_h = nullptr, *n_ecd = nullptr, *n_exs = nullptr,
           *n_ers = nullptr;
    long long* n_ioff = nullptr;
    auto undo = [&]() {
        (void)hipStreamSynchronize(c->stream);
        dfree(c, n_kind);
        dfree(c, n_inst);
        dfree(c, n_ngb);
        dfree(c, n_by);
        dfree(c, n_pos);
        dfree(c, n_pk);
        dfree(c, n_E);
        dfree(c, n_h);
        dfree(c, n_ecd);
        dfree(c, n_exs);
        dfree(c, n_ers);
        dfree(c, n_ioff);
    };
#define ATRY(x)                       \
    do {                              \
        rt_status s_ = (x);           \
        if (s_ != RT_OK) {            \
            undo();                   \
            return s_;                \
        }                             \
    } while (0)
    ATRY(upload(c, &n_kind, ek.data(), total));
    ATRY(upload(c, &n_inst, ei.data(), total));
    ATRY(upload(c, &n_pos, ep.data(), 3 * total));
    ATRY(upload(c, &n_pk, epk.data(), total * c->nf));
    ATRY(upload(c, &n_E, esrc.data(), static_cast<long long>(c->n_inst) * c->nf));
    ATRY(upload(c, &n_by, by_inst.data(), total));
    ATRY(upload(c, &n_ioff, ioff.data(), c->n_inst + 1ll));
    ATRY(alloc_n(c, &n_ngb, std::max<long long>(1, total) * c->K));
    ATRY(alloc_n(c, &n_h, std::max<long long>(1, total)));
    ATRY(alloc_n(c, &n_ecd, 3 * necd));
    ATRY(alloc_n(c, &n_exs, necd * c->nf));
    ATRY(alloc_n(c, &n_ers, necd * c->nf));
#undef ATRY
    // The captured forward steps refer to the emitters' buffers (virtual
    // particles of empty emission cones): drop them, and free the old buffers
    // once no queued work uses them.
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    dfree(c, c->em_kind);
    dfree(c, c->em_inst);
    dfree(c, c->em_pos);
    dfree(c, c->em_pk);
    dfree(c, c->E_src);
    dfree(c, c->em_ngb);
    dfree(c, c->em_h);
    dfree(c, c->ecd);
    dfree(c, c->exs);
    dfree(c, c->ers);
    dfree(c, c->em_by_inst);
    dfree(c, c->em_ioff);
    c->em_kind = n_kind;
    c->em_inst = n_inst;
    c->em_pos = n_pos;
    c->em_pk = n_pk;
    c->E_src = n_E;
    c->em_ngb = n_ngb;
    c->em_h = n_h;
    c->ecd = n_ecd;
    c->exs = n_exs;
    c->ers = n_ers;
    c->em_by_inst = n_by;
    c->em_ioff = n_ioff;
    c->n_emit = total;
    c->h_em_inst = ei;
    TRY(fill_f64(c, c->exs, necd * c->nf, 0.0));
    TRY(fill_f64(c, c->ers, necd * c->nf, 0.0));
    TRY(fill_f64(c, c->ecd, 3 * necd, 0.0));
    if (total > 0) {
        hipLaunchKernelGGL(k_knn, dim3(grid_for(total, 128)), dim3(128), 0, c->stream, total, c->em_pos, c->em_inst, 0,
                           c->grid_d, c->cell_start, c->cell_idx, c->pos, c->K, c->em_ngb, c->em_h);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RT_OK;
}
}  // namespace

rt_status rt_step(rt_ctx* c, int32_t n_steps) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    if (n_steps < 0) return fail(c, RT_EINVAL, "n_steps < 0");
    for (int k = 0; k < 8; ++k) c->tm[k] = 0.0;
    if (c->timing) HIPCHK(c, hipMemsetAsync(c->cnt + kCntBytes, 0, 2 * sizeof(long long), c->stream));
    bool hopcap = false;
    // a halt left by an error of the previous call
    hipLaunchKernelGGL(k_clear_halt, dim3(1), dim3(64), 0, c->stream, c->cnt);
    HIPCHK(c, hipGetLastError());
    for (int s = 0; s < n_steps;) {
        // whole-step graphs once the forward-step count is known and nothing
        // needs the host between forward steps (a tuning step, timing, a fixed
        // batch); while the tuner waits for a representative step, one step
        // per check
        const bool tune_pending = c->tune_mode < 0 && !c->tuned;
        const bool graphable = c->step_graphs_on && c->graphs_ok && !c->timing && c->p.hop_batch <= 0 && c->last_hops > 0 &&
                               !(tune_pending && (c->last_hops >= 16 || c->tune_mode == -2));
        int done = 0;
        if (graphable) TRY(graph_steps(c, tune_pending ? 1 : std::min(n_steps - s, 1024), &done, &hopcap));
        if (done == 0) {
            TRY(one_step(c, &hopcap));
            done = 1;
        }
        s += done;
        const long long flags = c->h_cnt[kCntFlags];
        if (flags & (kFlagVipOverflow | kFlagRecOverflow)) return fail(c, RT_EOVERFLOW, "work buffer overflow");
        if (flags & kFlagNonFinite) return fail(c, RT_ENONFINITE, "non-finite ledger");
        if (flags & kFlagDrift)
            return fail(c, RT_EDRIFT, "FP32 photons in flight drifted more than 1e-3 from the ledger: not rescaled");
    }
    if (hopcap) return fail(c, RT_EHOPCAP, "a step reached max_hops");
    return RT_OK;
}

rt_status rt_get_state(rt_ctx* c, double* x_HI, double* T, double* absorbed, double* passing, double* ledger,
                       int64_t* counters) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (x_HI) HIPCHK(c, hipMemcpy(x_HI, c->xHI, sizeof(double) * c->N, hipMemcpyDefault));
    if (T) HIPCHK(c, hipMemcpy(T, c->T, sizeof(double) * c->N, hipMemcpyDefault));
    if (absorbed) HIPCHK(c, hipMemcpy(absorbed, c->A, sizeof(double) * c->N * c->nf, hipMemcpyDefault));
    if (passing) HIPCHK(c, hipMemcpy(passing, c->P, sizeof(double) * c->N * c->nf, hipMemcpyDefault));
    if (ledger) HIPCHK(c, hipMemcpy(ledger, c->led, sizeof(double) * 5 * c->n_inst * c->nf, hipMemcpyDefault));
    if (counters) {
        long long h[kCntN];
        HIPCHK(c, hipMemcpy(h, c->cnt, sizeof(h), hipMemcpyDefault));
        counters[0] = h[kCntSteps];
        counters[1] = h[kCntHops];
        counters[2] = h[kCntVips];
        counters[3] = h[kCntUpdates];
    }
    return RT_OK;
}

}  // extern "C"

namespace {

// Arguments of a shell profile, checked before any device work (RT_EINVAL).
rt_status shell_profile_check(rt_ctx* c, int32_t inst, const double* center, const double* axis, double half_height,
                              double r_max, int32_t n_shells, double norm, double* prof) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    if (!center || !prof || inst < 0 || inst >= c->n_inst) return fail(c, RT_EINVAL, "shell profile: bad pointer or instance");
    if (n_shells < 1 || n_shells > kProfMaxShells || static_cast<long long>(n_shells) * c->nf > kProfMaxCells)
        return fail(c, RT_EINVAL, "shell profile: n_shells out of range");
    if (!(r_max > 0.0) || !(norm > 0.0) || !std::isfinite(r_max) || !std::isfinite(norm) || !std::isfinite(half_height) ||
        !std::isfinite(center[0]) || !std::isfinite(center[1]) || !std::isfinite(center[2]))
        return fail(c, RT_EINVAL, "shell profile: r_max, norm, half_height and center must be finite, r_max and norm > 0");
    if (axis) {
        const double a2 = axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2];
        if (!(a2 > 0.0) || !std::isfinite(a2))
            return fail(c, RT_EINVAL, "shell profile: the axis's squared length must be finite and nonzero");
    }
    return RT_OK;
}

// The profile of the passing photons Pd (device) binned into the histogram
// sum[n_shells*nf], cnt[n_shells] (device, cleared here by fill kernels), copied
// out and normalised.  Allocates nothing.
rt_status shell_profile_run(rt_ctx* c, int32_t inst, const double* Pd, const double* center, const double* axis,
                            double half_height, double r_max, int32_t n_shells, int32_t mean, double norm, double* sum,
                            unsigned long long* cnt_d, double* prof, int64_t* count) {
    const int ncell = n_shells * c->nf;
    TRY(fill_f64(c, sum, ncell, 0.0));
    TRY(fill_i32(c, reinterpret_cast<int*>(cnt_d), 2ll * n_shells, 0));
    ProfileArgs a{};
    a.pos = c->pos;
    a.P = Pd;
    a.j0 = c->inst_off[inst];
    a.j1 = c->inst_off[inst + 1];
    a.nf = c->nf;
    a.n_shells = n_shells;
    a.cyl = axis ? 1 : 0;
    a.c0 = center[0];
    a.c1 = center[1];
    a.c2 = center[2];
    if (axis) {
        a.a0 = axis[0];
        a.a1 = axis[1];
        a.a2 = axis[2];
    }
    a.half_height = half_height;
    a.r_max = r_max;
    a.dt = c->p.dt;
    a.sum = sum;
    a.cnt = cnt_d;
    // Workgroups: small instances get one per 256 particles (up to 128), large
    // ones one per 2048 (up to 256).  More would not help large instances: every
    // workgroup's flush adds into the same few cache lines, and those atomics
    // serialise.
    const long long n = a.j1 - a.j0;
    const unsigned grid = static_cast<unsigned>(std::max<long long>(
        1, std::min<long long>(256, std::max<long long>((n + 2047) / 2048, std::min<long long>(128, (n + 255) / 256)))));
    const size_t lds = sizeof(double) * ncell + sizeof(unsigned) * n_shells;
    hipLaunchKernelGGL(k_shell_profile, dim3(grid), dim3(kProfBlock), lds, c->stream, a);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unsigned long long cnt[kProfMaxShells];
    HIPCHK(c, hipMemcpy(prof, sum, sizeof(double) * ncell, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(cnt, cnt_d, sizeof(unsigned long long) * n_shells, hipMemcpyDeviceToHost));
    for (int k = 0; k < n_shells; ++k) {
        if (count) count[k] = static_cast<int64_t>(cnt[k]);
        for (int nu = 0; nu < c->nf; ++nu) {
            double v = prof[static_cast<long long>(k) * c->nf + nu];
            if (mean) v = cnt[k] > 0 ? v / static_cast<double>(cnt[k]) : 0.0;
            prof[static_cast<long long>(k) * c->nf + nu] = v / norm;
        }
    }
    return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_shell_profile(rt_ctx* c, int32_t inst, const double* passing, const double* center, const double* axis,
                           double half_height, double r_max, int32_t n_shells, int32_t mean, double norm, double* prof,
                           int64_t* count) {
    TRY(shell_profile_check(c, inst, center, axis, half_height, r_max, n_shells, norm, prof));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->prof_sum) TRY(alloc_n(c, &c->prof_sum, kProfMaxCells));
    if (!c->prof_cnt) TRY(alloc_n(c, &c->prof_cnt, kProfMaxShells));
    const double* Pd = c->P;
    if (passing) {
        if (!c->prof_in) TRY(alloc_n(c, &c->prof_in, c->N * c->nf));
        HIPCHK(c, hipMemcpy(c->prof_in, passing, sizeof(double) * c->N * c->nf, hipMemcpyHostToDevice));
        Pd = c->prof_in;
    }
    return shell_profile_run(c, inst, Pd, center, axis, half_height, r_max, n_shells, mean, norm, c->prof_sum,
                             c->prof_cnt, prof, count);
}

rt_status rt_shell_profile_noalloc(rt_ctx* c, int32_t inst, const double* passing_dev, const double* center,
                                   const double* axis, double half_height, double r_max, int32_t n_shells,
                                   int32_t mean, double norm, double* prof, int64_t* count) {
    TRY(shell_profile_check(c, inst, center, axis, half_height, r_max, n_shells, norm, prof));
    const double* Pd = c->P;
    if (passing_dev) {
        hipPointerAttribute_t at{};
        const hipError_t e = hipPointerGetAttributes(&at, passing_dev);
        if (e != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)) {
            (void)hipGetLastError();
            return fail(c, RT_EINVAL, "shell profile (no allocation): passing must be device memory or NULL");
        }
        Pd = passing_dev;
    }
    TRY(resolve_scratch(c));
    unsigned char* base = static_cast<unsigned char*>(g_scratch[c->dev]);
    double* sum = reinterpret_cast<double*>(base);
    unsigned long long* cnt_d = reinterpret_cast<unsigned long long*>(base + sizeof(double) * kProfMaxCells);
    return shell_profile_run(c, inst, Pd, center, axis, half_height, r_max, n_shells, mean, norm, sum, cnt_d, prof,
                             count);
}

rt_status rt_set_barrier(rt_ctx* c, int32_t inst, const double* center, double radius) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    if (inst < 0 || inst >= c->n_inst || (radius > 0.0 && !center) || !(radius >= 0.0) || !std::isfinite(radius))
        return fail(c, RT_EINVAL, "barrier: bad instance, centre or radius");
    if (radius > 0.0)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(center[a])) return fail(c, RT_EINVAL, "barrier: centre must be finite");
    for (int a = 0; a < 3; ++a) c->bar[4 * inst + a] = radius > 0.0 ? center[a] : 0.0;
    c->bar[4 * inst + 3] = radius;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);  // the forward steps' kernel variant and arguments follow the barrier
    c->any_bar = false;
    for (int k = 0; k < c->n_inst; ++k) c->any_bar = c->any_bar || c->bar[4 * k + 3] > 0.0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->bar_d, c->bar.data(), sizeof(double) * c->bar.size(), hipMemcpyHostToDevice));
    if (c->f32)
        hipLaunchKernelGGL(k_barrier_edges<float4>, dim3(grid_for(c->N, 256)), dim3(256), 0, c->stream, c->N, c->pos,
                           c->rev_off, c->rev_ik, c->inst_of, c->bar_d, static_cast<float4*>(c->rev_v));
    else
        hipLaunchKernelGGL(k_barrier_edges<double4>, dim3(grid_for(c->N, 256)), dim3(256), 0, c->stream, c->N, c->pos,
                           c->rev_off, c->rev_ik, c->inst_of, c->bar_d, static_cast<double4*>(c->rev_v));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RT_OK;
}

rt_status rt_get_bins(rt_ctx* c, double* N, double* dir, double* clock) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long B = c->B;
    std::vector<double> U(c->n_inst);
    std::vector<int> inst_of(c->N);
    HIPCHK(c, hipMemcpy(inst_of.data(), c->inst_of, sizeof(int) * c->N, hipMemcpyDeviceToHost));
    if (c->f32) {
        std::vector<Bin4<float>> pk(B);
        std::vector<float> pc(B);
        HIPCHK(c, hipMemcpy(pk.data(), c->pk, sizeof(Bin4<float>) * B, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(pc.data(), c->pcl, sizeof(float) * B, hipMemcpyDeviceToHost));
        for (long long b = 0; b < B; ++b) {
            const int k = inst_of[b / c->G];
            if (N) N[b] = static_cast<double>(pk[b].n) * c->U[k];
            if (dir) {
                dir[3 * b] = pk[b].x;
                dir[3 * b + 1] = pk[b].y;
                dir[3 * b + 2] = pk[b].z;
            }
            if (clock) clock[b] = static_cast<double>(pc[b]) * c->p.dt;
        }
    } else {
        std::vector<Bin4<double>> pk(B);
        std::vector<double> pc(B);
        HIPCHK(c, hipMemcpy(pk.data(), c->pk, sizeof(Bin4<double>) * B, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(pc.data(), c->pcl, sizeof(double) * B, hipMemcpyDeviceToHost));
        for (long long b = 0; b < B; ++b) {
            if (N) N[b] = pk[b].n;
            if (dir) {
                dir[3 * b] = pk[b].x;
                dir[3 * b + 1] = pk[b].y;
                dir[3 * b + 2] = pk[b].z;
            }
            if (clock) clock[b] = pc[b];
        }
    }
    return RT_OK;
}

rt_status rt_get_neighbours(rt_ctx* c, int32_t* ngb, double* h) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (ngb) HIPCHK(c, hipMemcpy(ngb, c->ngb, sizeof(int) * c->N * c->K, hipMemcpyDeviceToHost));
    if (h) HIPCHK(c, hipMemcpy(h, c->h, sizeof(double) * c->N, hipMemcpyDeviceToHost));
    return RT_OK;
}

int64_t rt_n_emitters(const rt_ctx* c) { return c ? c->n_emit : 0; }

rt_status rt_get_emitter_neighbours(rt_ctx* c, int32_t* ngb, double* h) {
    if (!c) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->n_emit == 0) return RT_OK;
    if (ngb) HIPCHK(c, hipMemcpy(ngb, c->em_ngb, sizeof(int) * c->n_emit * c->K, hipMemcpyDeviceToHost));
    if (h) HIPCHK(c, hipMemcpy(h, c->em_h, sizeof(double) * c->n_emit, hipMemcpyDeviceToHost));
    return RT_OK;
}

rt_status rt_get_cone_masks(rt_ctx* c, uint64_t* mask) {
    if (!c || !mask) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // a mask is kept for every packet that became active; report those of the
    // packets still active (in flight after the last forward step)
    const long long B = c->B;
    HIPCHK(c, hipMemcpy(mask, c->cm, sizeof(uint64_t) * B, hipMemcpyDeviceToHost));
    const double lim = c->f32 ? 1.0 : c->p.dt;
    std::vector<double> n(B), clk(B);
    if (c->f32) {
        std::vector<Bin4<float>> pk(B);
        std::vector<float> pc(B);
        HIPCHK(c, hipMemcpy(pk.data(), c->pk, sizeof(Bin4<float>) * B, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(pc.data(), c->pcl, sizeof(float) * B, hipMemcpyDeviceToHost));
        for (long long b = 0; b < B; ++b) {
            n[b] = pk[b].n;
            clk[b] = pc[b];
        }
    } else {
        std::vector<Bin4<double>> pk(B);
        HIPCHK(c, hipMemcpy(pk.data(), c->pk, sizeof(Bin4<double>) * B, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(clk.data(), c->pcl, sizeof(double) * B, hipMemcpyDeviceToHost));
        for (long long b = 0; b < B; ++b) n[b] = pk[b].n;
    }
    for (long long b = 0; b < B; ++b)
        if (!(n[b] > 0.0 && clk[b] < lim)) mask[b] = 0;
    return RT_OK;
}

rt_status rt_get_pending_rr(rt_ctx* c, double* nrr) {
    if (!c || !nrr) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(nrr, c->nrr[c->nrr_cur], sizeof(double) * c->N, hipMemcpyDeviceToHost));
    return RT_OK;
}

rt_status rt_set_timing(rt_ctx* c, int32_t on) {
    if (!c) return RT_EINVAL;
    c->timing = on != 0;
    return RT_OK;
}

rt_status rt_get_timing(rt_ctx* c, double* out, int32_t n) {
    if (!c || !out || n < 0) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    long long h[kCntN];
    HIPCHK(c, hipMemcpy(h, c->cnt, sizeof(h), hipMemcpyDeviceToHost));
    // Dense model of one forward step, for comparison: every slot's packet and
    // clock read and written; per edge its sender word and inbox read and its
    // inbox written; per particle and bin A and P read and written.
    const double rsz = c->f32 ? 4.0 : 8.0, isz = c->dl64 ? 16.0 : 8.0;
    const double dense = 2.0 * 5.0 * rsz * static_cast<double>(c->B) +
                         (c->K * (4.0 + 2.0 * isz) + 2.0 * 2.0 * 8.0 * c->nf) * static_cast<double>(c->N);
    double v[9] = {c->tm[0], c->tm[1], c->tm[2], c->tm[3], c->tm[4], c->tm[5], static_cast<double>(h[kCntBytes]),
                   static_cast<double>(h[kCntTiles]), dense};
    for (int k = 0; k < n && k < 9; ++k) out[k] = v[k];
    return RT_OK;
}

rt_status rt_set_step_graphs(rt_ctx* c, int32_t on) {
    if (!c || (on != 0 && on != 1)) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    c->step_graphs_on = on != 0;
    return RT_OK;
}

rt_status rt_set_hop_shape(rt_ctx* c, int32_t shape) {
    if (!c || shape < -2 || shape >= kHopShapes) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->tune_mode = shape;
    if (shape >= 0) {
        c->hop_shape = shape;
        c->tuned = true;
    } else {
        c->hop_shape = 0;
        c->tuned = false;
        c->tune_steps_left = kTuneShapes;
        for (int k = 0; k < kHopShapes; ++k) {
            c->tune_ms[k] = 0.0;
            c->tune_n[k] = 0;
        }
    }
    return RT_OK;
}

rt_status rt_get_hop_shape(rt_ctx* c, int32_t* shape, int32_t* tuned, double* ms_per_launch) {
    if (!c) return RT_EINVAL;
    if (shape) *shape = c->hop_shape;
    if (tuned) *tuned = (c->tuned && c->tune_mode < 0) ? 1 : 0;
    if (ms_per_launch)
        for (int k = 0; k < kHopShapes; ++k) ms_per_launch[k] = c->tune_n[k] ? c->tune_ms[k] / c->tune_n[k] : 0.0;
    return RT_OK;
}

namespace {
struct BlobHeader {
    long long magic, N, B, nf, n_inst, f32, step, serial, last_hops;
};
}  // namespace

rt_status rt_get_state_blob(rt_ctx* c, void* blob, size_t* bytes) {
    if (!c || !bytes) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    const size_t rsz = c->f32 ? 4 : 8;
    const size_t need = sizeof(BlobHeader) + 5 * rsz * c->B + 3 * 8 * c->N + 8 * 5 * c->n_inst * c->nf +
                        8 * c->n_inst * c->nf + 8 * kCntN;
    if (!blob) {
        *bytes = need;
        return RT_OK;
    }
    if (*bytes < need) return fail(c, RT_ESTATE, "blob too small");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    char* q = static_cast<char*>(blob);
    // the stamp counter and the last step's forward-step count travel too, so
    // that a restored context numbers and batches its forward steps as the
    // original would have
    BlobHeader hd{0x54524150ll, c->N, c->B, c->nf, c->n_inst, c->f32, c->step, c->serial, c->last_hops};
    std::memcpy(q, &hd, sizeof hd);
    q += sizeof hd;
    HIPCHK(c, hipMemcpy(q, c->pk, 4 * rsz * c->B, hipMemcpyDeviceToHost));
    q += 4 * rsz * c->B;
    HIPCHK(c, hipMemcpy(q, c->pcl, rsz * c->B, hipMemcpyDeviceToHost));
    q += rsz * c->B;
    HIPCHK(c, hipMemcpy(q, c->xHI, 8 * c->N, hipMemcpyDeviceToHost));
    q += 8 * c->N;
    HIPCHK(c, hipMemcpy(q, c->T, 8 * c->N, hipMemcpyDeviceToHost));
    q += 8 * c->N;
    HIPCHK(c, hipMemcpy(q, c->nrr[c->nrr_cur], 8 * c->N, hipMemcpyDeviceToHost));
    q += 8 * c->N;
    HIPCHK(c, hipMemcpy(q, c->led, 8 * 5 * c->n_inst * c->nf, hipMemcpyDeviceToHost));
    q += 8 * 5 * c->n_inst * c->nf;
    HIPCHK(c, hipMemcpy(q, c->scale, 8 * c->n_inst * c->nf, hipMemcpyDeviceToHost));
    q += 8 * c->n_inst * c->nf;
    HIPCHK(c, hipMemcpy(q, c->cnt, 8 * kCntN, hipMemcpyDeviceToHost));
    {  // the byte and tile tallies are timing diagnostics, not state
        long long* cq = reinterpret_cast<long long*>(q);
        cq[kCntBytes] = 0;
        cq[kCntTiles] = 0;
    }
    *bytes = need;
    return RT_OK;
}

rt_status rt_set_state_blob(rt_ctx* c, const void* blob, size_t bytes) {
    if (!c || !blob) return RT_EINVAL;
    if (c->sticky) return RT_EDEVICE;
    size_t need = 0;
    TRY(rt_get_state_blob(c, nullptr, &need));
    if (bytes != need) return fail(c, RT_ESTATE, "blob size mismatch");
    BlobHeader hd;
    std::memcpy(&hd, blob, sizeof hd);
    if (hd.magic != 0x54524150ll || hd.N != c->N || hd.B != c->B || hd.nf != c->nf || hd.n_inst != c->n_inst ||
        hd.f32 != (c->f32 ? 1 : 0))
        return fail(c, RT_ESTATE, "blob from a different context");
    const size_t rsz = c->f32 ? 4 : 8;
    const char* q = static_cast<const char*>(blob) + sizeof hd;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nrr_cur = 0;
    HIPCHK(c, hipMemcpy(c->pk, q, 4 * rsz * c->B, hipMemcpyHostToDevice));
    q += 4 * rsz * c->B;
    HIPCHK(c, hipMemcpy(c->pcl, q, rsz * c->B, hipMemcpyHostToDevice));
    q += rsz * c->B;
    HIPCHK(c, hipMemcpy(c->xHI, q, 8 * c->N, hipMemcpyHostToDevice));
    q += 8 * c->N;
    HIPCHK(c, hipMemcpy(c->T, q, 8 * c->N, hipMemcpyHostToDevice));
    if (c->rc3) {  // the restored temperatures' rate coefficients
        hipLaunchKernelGGL(k_rates_cache, dim3(grid_for(c->N, 256)), dim3(256), 0, c->stream, c->N, c->T, c->rc3);
        HIPCHK(c, hipGetLastError());
    }
    q += 8 * c->N;
    HIPCHK(c, hipMemcpy(c->nrr[0], q, 8 * c->N, hipMemcpyHostToDevice));
    q += 8 * c->N;
    HIPCHK(c, hipMemcpy(c->led, q, 8 * 5 * c->n_inst * c->nf, hipMemcpyHostToDevice));
    q += 8 * 5 * c->n_inst * c->nf;
    HIPCHK(c, hipMemcpy(c->scale, q, 8 * c->n_inst * c->nf, hipMemcpyHostToDevice));
    q += 8 * c->n_inst * c->nf;
    HIPCHK(c, hipMemcpy(c->cnt, q, 8 * kCntN, hipMemcpyHostToDevice));
    c->step = hd.step;
    c->serial = hd.serial;
    c->last_hops = hd.last_hops;
    for (int b = 0; b < 2; ++b) {  // forget the marks of this context's own earlier steps
        HIPCHK(c, hipMemsetAsync(c->inbox[b], 0xff, c->inbox_bytes, c->stream));
        TRY(fill_i32(c, c->hot[b], c->hot_len, -1));
    }
    TRY(fill_i32(c, c->rest, c->ntiles, 1));  // the restored bins: every tile runs at the next hop 0
    c->rest_unknown = true;
    if (c->f32) {
        hipLaunchKernelGGL(k_kappa_init, dim3(grid_for(c->N, 256)), dim3(256), 0, c->stream, c->N, c->xHI, c->nH,
                           c->L_d, c->inst_of, c->kappa);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RT_OK;
}

void rt_destroy(rt_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto& b : c->owned) {
        if (c->p.dealloc)
            c->p.dealloc(c->p.alloc_user, b.p);
        else if (!c->p.alloc)
            (void)hipFree(b.p);
    }
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    if (c->h_listlen) (void)hipHostFree(c->h_listlen);
    delete c;
}

}  // extern "C"
