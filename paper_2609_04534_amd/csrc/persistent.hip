// Single-launch kernels over all groups of a plan (batches of uneven
// degree).
//
// Every group is a segment of work tiles: 64 blocks per tile for the
// lane-per-block body and BPW blocks per tile for the wave-per-tile body.
// A work item is `tpw` consecutive tiles of one segment; the items of all
// segments, in the configured segment order, form one list.  apply and
// apply_inverse launch one one-wave workgroup per item of that list, which
// finds its segment by a scan of the (few) segment starts and runs the
// group's tile body, inlined per degree (no calls, no scratch; each switch
// branch has its own registers).  The solve runs a grid whose workgroups
// walk the item list with the grid stride, so its per-workgroup summaries
// fit the plan's partials.  No counters or atomics: the launch is
// capturable in a HIP graph, and since each tile's arithmetic does not
// depend on which workgroup runs it, its results are bitwise those of the
// per-group launches with the same tile bodies.  Factor tables are loaded
// once per workgroup (per item).
//
// The body, tiles per item, segment order and solve grid are kept per call
// and dtype (Plan::pcfg); tp_plan_autotune times the alternatives.
#include <algorithm>
#include <climits>
#include <vector>

#include "eo.h"
#include "lane.h"

namespace tpfdm {

struct PSeg {
    const double* h;
    int64_t nblocks;
    int64_t offset;
    int64_t block0;
    int64_t tiles;        // tiles of the segment's body (64 blocks for lane, BPW for wave)
    int64_t first_item;   // first work item of the segment in the launch
    int32_t logB;
    int32_t n;
    int32_t lane;         // lane-per-block body (n <= 4; never in the solve)
    int32_t tpw;          // tiles per work item
};

namespace {

constexpr int kMaxSlab = Slab<8>::BPW * Slab<8>::size;  // largest BPW * slab size over n <= 8

template <int N>
constexpr size_t solve_lds_bytes() {
    return sizeof(SolveLdsR<N>) + 64 * sizeof(double) + 64 * sizeof(double);
}
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kSolveLdsBytes =
    cmax(cmax(cmax(solve_lds_bytes<2>(), solve_lds_bytes<3>()), cmax(solve_lds_bytes<4>(), solve_lds_bytes<5>())),
         cmax(cmax(solve_lds_bytes<6>(), solve_lds_bytes<7>()), solve_lds_bytes<8>()));

__device__ __forceinline__ const char* dev_table(const char* base, int n, int tab, int et) {
    return base + static_cast<size_t>(((n * EO_NTAB + tab) * 2 + et) * kEOSlot) * sizeof(double);
}

__device__ __forceinline__ GArgs seg_args(const PSeg& sg) {
    GArgs a;
    a.h = sg.h;
    a.nblocks = sg.nblocks;
    a.offset = sg.offset;
    a.logB = sg.logB;
    return a;
}

// ------------------------------------------------------------ apply
template <int N, typename TS, typename TC, bool NT>
__device__ __forceinline__ void seg_apply_lane(const TS* __restrict__ u, TS* __restrict__ v, const PSeg& sg,
                                               const TC* __restrict__ ptab, int64_t t0, int64_t t1) {
    Pair<N, TC> R;
#pragma unroll
    for (int i = 0; i < N * N; ++i) {
        R.m[i] = ptab[i];
        R.p[i] = ptab[N * N + i];
    }
    const int lb = sg.logB;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t g = t * 64 + threadIdx.x;
        if (g >= sg.nblocks) continue;
        const int64_t base = sg.offset + block_base(g, lb, N * N * N);
        const TS* ub = u + base;
        TS* vb = v + base;
        TC sx, sy, sz;
        block_scales(sg.h, g, sx, sy, sz);
        TC acc[N * N * N];
        lane_apply<N, TC>([&](int q) { return ldv<NT, TC>(ub + (static_cast<int64_t>(q) << lb)); }, R, sx, sy, sz, acc);
#pragma unroll
        for (int q = 0; q < N * N * N; ++q) stv<NT>(vb + (static_cast<int64_t>(q) << lb), acc[q]);
    }
}

template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void seg_apply_wave(const TS* __restrict__ u, TS* __restrict__ v, const PSeg& sg,
                                               const TC* __restrict__ tab, TC* s1, TC* s2, TC* stab, int64_t t0,
                                               int64_t t1) {
    using L = Slab<N>;
    ApplyTab<N, TC> A;
    table_to_regs(A.v, tab, stab, ApplyTab<N, TC>::COUNT);
    const GArgs G = seg_args(sg);
    const int lane = threadIdx.x;
    const int lw = lane / L::N2;
    const int lp = lane - lw * L::N2;
    const int li = lp / N, lj = lp - (lp / N) * N;
    const int so = (lw < L::BPW ? lw : 0) * L::size;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of<N>(G, t);
        const Pencil<N> pc(nvalid);
        TC x[N];
        if (lw < L::BPW && lw < nvalid) pencil_load<N, VP>(x, pencil_ptr<N>(u, G, g0 + lw, li, lj), G.logB);
        TC sx = TC(1), sy = TC(1), sz = TC(1);
        if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
        eo_apply_body<N>(pc, x, v, G, g0, s1 + so, s2 + so, A.ME(), A.MO(), A.PE(), A.PO(), sx, sy, sz);
    }
}

template <int N, typename TS, typename TC>
__device__ __forceinline__ void seg_apply(const TS* u, TS* v, const PSeg& sg, const char* tabs, int op, bool vp,
                                          TC* lds, int64_t t0, int64_t t1) {
    const int et = sizeof(TC) == 8 ? 0 : 1;
    if constexpr (N <= kLaneMaxN) {
        if (sg.lane) {
            const TC* pt =
                reinterpret_cast<const TC*>(dev_table(tabs, N, op == TP_OP_CELL ? EO_PLAIN_A : EO_PLAIN_K, et));
            if ((static_cast<int64_t>(sizeof(TS)) << sg.logB) >= 128)
                seg_apply_lane<N, TS, TC, true>(u, v, sg, pt, t0, t1);
            else
                seg_apply_lane<N, TS, TC, false>(u, v, sg, pt, t0, t1);
            return;
        }
    }
    const TC* tab = reinterpret_cast<const TC*>(dev_table(tabs, N, op == TP_OP_CELL ? EO_APPLY_A : EO_APPLY_K, et));
    if (vp)
        seg_apply_wave<N, true>(u, v, sg, tab, lds, lds + kMaxSlab, lds + 2 * kMaxSlab, t0, t1);
    else
        seg_apply_wave<N, false>(u, v, sg, tab, lds, lds + kMaxSlab, lds + 2 * kMaxSlab, t0, t1);
}

// ------------------------------------------------------------ inverse
template <int N, typename TS, typename TC, bool NT>
__device__ __forceinline__ void seg_inverse_lane(const TS* __restrict__ r, TS* __restrict__ x, const PSeg& sg,
                                                 const TC* __restrict__ ptab, int64_t t0, int64_t t1) {
    Eig<N, TC> E;
#pragma unroll
    for (int i = 0; i < N * N; ++i) E.s[i] = ptab[i];
#pragma unroll
    for (int i = 0; i < N; ++i) E.lam[i] = ptab[N * N + i];
    const int lb = sg.logB;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t g = t * 64 + threadIdx.x;
        if (g >= sg.nblocks) continue;
        const int64_t base = sg.offset + block_base(g, lb, N * N * N);
        const TS* rb = r + base;
        TS* xb = x + base;
        TC sx, sy, sz;
        block_scales(sg.h, g, sx, sy, sz);
        TC v[N * N * N];
#pragma unroll
        for (int q = 0; q < N * N * N; ++q) v[q] = ldv<NT, TC>(rb + (static_cast<int64_t>(q) << lb));
        lane_fdm_inplace<N, TC>(v, E, sx, sy, sz);
#pragma unroll
        for (int q = 0; q < N * N * N; ++q) stv<NT>(xb + (static_cast<int64_t>(q) << lb), v[q]);
    }
}

template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void seg_inverse_wave(const TS* __restrict__ r, TS* __restrict__ x, const PSeg& sg,
                                                 const TC* __restrict__ tab, TC* s1, TC* stab, int64_t t0,
                                                 int64_t t1) {
    using L = Slab<N>;
    using S = EOShape<N>;
    InvTab<N, TC> I;
    table_to_regs(I.v, tab, stab, S::SE + S::SO + N);
    const TC* lam = stab + S::SE + S::SO;
    const GArgs G = seg_args(sg);
    const int lane = threadIdx.x;
    const int lw = lane / L::N2;
    const int lp = lane - lw * L::N2;
    const int li = lp / N, lj = lp - (lp / N) * N;
    const int so = (lw < L::BPW ? lw : 0) * L::size;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of<N>(G, t);
        const Pencil<N> pc(nvalid);
        TC xin[N];
        if (lw < L::BPW && lw < nvalid) pencil_load<N, VP>(xin, pencil_ptr<N>(r, G, g0 + lw, li, lj), G.logB);
        TC sx = TC(1), sy = TC(1), sz = TC(1);
        if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
        eo_inverse_body<N, VP>(pc, xin, x, G, g0, s1 + so, I.SE(), I.SO(), lam, sx, sy, sz);
    }
}

template <int N, typename TS, typename TC>
__device__ __forceinline__ void seg_inverse(const TS* r, TS* x, const PSeg& sg, const char* tabs, bool vp, TC* lds,
                                            int64_t t0, int64_t t1) {
    const int et = sizeof(TC) == 8 ? 0 : 1;
    if constexpr (N <= kLaneMaxN) {
        if (sg.lane) {
            const TC* pt = reinterpret_cast<const TC*>(dev_table(tabs, N, EO_PLAIN_S, et));
            if ((static_cast<int64_t>(sizeof(TS)) << sg.logB) >= 128)
                seg_inverse_lane<N, TS, TC, true>(r, x, sg, pt, t0, t1);
            else
                seg_inverse_lane<N, TS, TC, false>(r, x, sg, pt, t0, t1);
            return;
        }
    }
    const TC* tab = reinterpret_cast<const TC*>(dev_table(tabs, N, EO_INV, et));
    if (vp)
        seg_inverse_wave<N, true>(r, x, sg, tab, lds, lds + kMaxSlab, t0, t1);
    else
        seg_inverse_wave<N, false>(r, x, sg, tab, lds, lds + kMaxSlab, t0, t1);
}

// ------------------------------------------------------------ solve
template <int N, typename TI, int RND>
__device__ __forceinline__ void seg_solve(const double* b, double* x, const PSeg& sg, const char* tabs, char* lds,
                                          int64_t t0, int64_t t1, double rtol, int maxit, int32_t* iters,
                                          double* relres, SolveAcc& acc) {
    using S = EOShape<N>;
    SolveLdsR<N>& L = *reinterpret_cast<SolveLdsR<N>*>(lds);
    TI* stabS = reinterpret_cast<TI*>(lds + sizeof(SolveLdsR<N>));
    // 1D tables read at wave-uniform addresses (scalar loads), the
    // eigenvalues through LDS (as in the per-group solve kernel)
    const double* tA = reinterpret_cast<const double*>(dev_table(tabs, N, EO_APPLY_A, 0));
    const TI* tS = reinterpret_cast<const TI*>(dev_table(tabs, N, EO_INV, sizeof(TI) == 8 ? 0 : 1));
    stage_table<TI, S::SE + S::SO + N>(tS, stabS);
    const TI* lam = stabS + S::SE + S::SO;
    const GArgs G = seg_args(sg);
    for (int64_t t = t0; t < t1; ++t)
        eo_solve_tile<N, TI, RND, false>(b, x, G, t * Slab<N>::BPW, nvalid_of<N>(G, t), L, tA, tS, lam, rtol,
                                         maxit, iters, relres, sg.block0, acc);
}




// Segment of work item w: segments in launch order, each covering the items
// [first_item, first_item + ceil(tiles / tpw)) of the launch.
__device__ __forceinline__ int flat_segment(const PSeg* __restrict__ segs, int nseg, int64_t w) {
    int si = 0;
    while (si + 1 < nseg && segs[si + 1].first_item <= w) ++si;
    return si;
}

__device__ __forceinline__ void item_tiles(const PSeg& sg, int64_t w, int64_t& t0, int64_t& t1) {
    t0 = (w - sg.first_item) * sg.tpw;
    t1 = t0 + sg.tpw < sg.tiles ? t0 + sg.tpw : sg.tiles;
}

// One launch over all groups: one workgroup per work item, the group's body
// inlined per degree (no calls, no scratch).  Every item is independent, so
// the hardware dispatcher balances the mix.
template <typename TS, typename TC>
__global__ __launch_bounds__(64, 2) void k_persist_apply(const TS* __restrict__ u, TS* __restrict__ v,
                                                         const PSeg* __restrict__ segs, int nseg,
                                                         const char* __restrict__ tabs, int op,
                                                         unsigned long long vpmask) {
    __shared__ __align__(16) TC lds[2 * kMaxSlab + 64];
    const int si = flat_segment(segs, nseg, blockIdx.x);
    const PSeg sg = segs[si];
    int64_t t0, t1;
    item_tiles(sg, blockIdx.x, t0, t1);
    const bool vp = si < 64 && ((vpmask >> si) & 1ull);
    switch (sg.n) {
        case 2: seg_apply<2, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        case 3: seg_apply<3, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        case 4: seg_apply<4, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        case 5: seg_apply<5, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        case 6: seg_apply<6, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        case 7: seg_apply<7, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        case 8: seg_apply<8, TS, TC>(u, v, sg, tabs, op, vp, lds, t0, t1); break;
        default: break;
    }
}

template <typename TS, typename TC>
__global__ __launch_bounds__(64, 2) void k_persist_inverse(const TS* __restrict__ r, TS* __restrict__ x,
                                                           const PSeg* __restrict__ segs, int nseg,
                                                           const char* __restrict__ tabs, unsigned long long vpmask) {
    __shared__ __align__(16) TC lds[kMaxSlab + 64];
    const int si = flat_segment(segs, nseg, blockIdx.x);
    const PSeg sg = segs[si];
    int64_t t0, t1;
    item_tiles(sg, blockIdx.x, t0, t1);
    const bool vp = si < 64 && ((vpmask >> si) & 1ull);
    switch (sg.n) {
        case 2: seg_inverse<2, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        case 3: seg_inverse<3, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        case 4: seg_inverse<4, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        case 5: seg_inverse<5, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        case 6: seg_inverse<6, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        case 7: seg_inverse<7, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        case 8: seg_inverse<8, TS, TC>(r, x, sg, tabs, vp, lds, t0, t1); break;
        default: break;
    }
}

// The solve over all groups: workgroups walk the item list with the grid
// stride, the group's body inlined per degree.
template <typename TI, int RND>
__global__ __launch_bounds__(64, 2) void k_persist_solve(const double* __restrict__ b, double* __restrict__ x,
                                                         const PSeg* __restrict__ segs, int nseg,
                                                         const char* __restrict__ tabs, double rtol, int maxit,
                                                         int32_t* __restrict__ iters, double* __restrict__ relres,
                                                         int64_t total, SolvePartial* parts) {
    __shared__ __align__(16) char lds[kSolveLdsBytes];
    SolveAcc acc;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const PSeg sg = segs[flat_segment(segs, nseg, w)];
        int64_t t0, t1;
        item_tiles(sg, w, t0, t1);
        switch (sg.n) {
            case 2: seg_solve<2, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            case 3: seg_solve<3, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            case 4: seg_solve<4, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            case 5: seg_solve<5, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            case 6: seg_solve<6, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            case 7: seg_solve<7, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            case 8: seg_solve<8, TI, RND>(b, x, sg, tabs, lds, t0, t1, rtol, maxit, iters, relres, acc); break;
            default: break;
        }
    }
    acc.flush(parts + blockIdx.x);
}

int bpw_of(int n) { return n * n >= 64 ? 1 : 64 / (n * n); }

int64_t seg_tiles(const GroupInfo& g, bool lane) {
    return lane ? (g.nblocks + 63) / 64 : (g.nblocks + bpw_of(g.n) - 1) / bpw_of(g.n);
}

const PSeg* seg_table(const Plan& plan, int call, int dt) {
    return static_cast<const PSeg*>(plan.segs_dev) + static_cast<size_t>(call * 4 + dt) * plan.groups.size();
}

// Vector pencils per segment in launch order (bit i for segment i < 64).
unsigned long long vp_mask(const Plan& plan, const PersistCfg& c, const void* a, const void* b, int esize) {
    unsigned long long m = 0;
    const int vec = 16 / esize;
    for (size_t i = 0; i < c.order.size() && i < 64; ++i) {
        const GroupInfo& g = plan.groups[c.order[i]];
        if (g.logB != 0 || g.n % vec != 0) continue;
        const uintptr_t pa = reinterpret_cast<uintptr_t>(a) + static_cast<uintptr_t>(g.offset) * esize;
        const uintptr_t pb = reinterpret_cast<uintptr_t>(b) + static_cast<uintptr_t>(g.offset) * esize;
        if (pa % 16 == 0 && pb % 16 == 0) m |= 1ull << i;
    }
    return m;
}

int64_t occupancy_grid(const Plan& plan, const void* kern) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, 0) != hipSuccess || occ <= 0) occ = 8;
    return static_cast<int64_t>(plan.cus) * occ;
}

tp_status check_p(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <typename TS, typename TC>
tp_status papply(const Plan& plan, int dt, int op, const void* u, void* v, hipStream_t s) {
    const PersistCfg& c = plan.pcfg[PCALL_APPLY][dt];
    if (c.items <= 0) return TP_OK;   // one workgroup per item
    hipLaunchKernelGGL((k_persist_apply<TS, TC>), dim3(static_cast<unsigned>(c.items)), dim3(64), 0, s,
                       static_cast<const TS*>(u), static_cast<TS*>(v), seg_table(plan, PCALL_APPLY, dt),
                       static_cast<int>(plan.groups.size()), static_cast<const char*>(plan.eo_dev), op,
                       vp_mask(plan, c, u, v, sizeof(TS)));
    return check_p("persistent apply launch");
}

template <typename TS, typename TC>
tp_status pinverse(const Plan& plan, int dt, const void* r, void* x, hipStream_t s) {
    const PersistCfg& c = plan.pcfg[PCALL_INVERSE][dt];
    if (c.items <= 0) return TP_OK;
    hipLaunchKernelGGL((k_persist_inverse<TS, TC>), dim3(static_cast<unsigned>(c.items)), dim3(64), 0, s,
                       static_cast<const TS*>(r), static_cast<TS*>(x), seg_table(plan, PCALL_INVERSE, dt),
                       static_cast<int>(plan.groups.size()), static_cast<const char*>(plan.eo_dev),
                       vp_mask(plan, c, r, x, sizeof(TS)));
    return check_p("persistent apply_inverse launch");
}

template <typename TI, int RND>
tp_status psolve(const Plan& plan, int dt, const double* b, double* x, double rtol, int maxit, int32_t* iters,
                 double* relres, const SolveWork& w, int64_t* nparts, hipStream_t s) {
    const PersistCfg& c = plan.pcfg[PCALL_SOLVE][dt];
    if (c.items <= 0) return TP_OK;
    const void* kern = reinterpret_cast<const void*>(&k_persist_solve<TI, RND>);
    static int occ_per_cu = 0;   // the kernel's resident workgroups per CU (a property of the code object)
    if (occ_per_cu == 0) occ_per_cu = static_cast<int>(occupancy_grid(plan, kern) / plan.cus);
    const int64_t occ = static_cast<int64_t>(plan.cus) * occ_per_cu;
    const int64_t want = c.grid == 0 ? c.items : c.grid == 2 ? std::max<int64_t>(1, occ / 2) : occ;
    const int64_t grid = std::max<int64_t>(1, std::min(want, c.items));
    if (grid > w.cap) return set_error(TP_ERR_UNSUPPORTED, "too many solve workgroups");
    *nparts = grid;
    hipLaunchKernelGGL((k_persist_solve<TI, RND>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b, x,
                       seg_table(plan, PCALL_SOLVE, dt), static_cast<int>(plan.groups.size()),
                       static_cast<const char*>(plan.eo_dev), rtol, maxit, iters, relres, c.items,
                       w.parts);
    return check_p("persistent solve launch");
}

}  // namespace

bool persistent_lane_ok(const Plan& plan, const GroupInfo& g) {
    (void)plan;
    return g.n <= kLaneMaxN;
}

tp_status persistent_upload(Plan& plan, int call, int dt) {
    const size_t ng = plan.groups.size();
    PersistCfg& c = plan.pcfg[call][dt];
    std::vector<PSeg> segs;
    int64_t first = 0;
    for (size_t k = 0; k < ng; ++k) {
        const int gi = c.order[k];
        const GroupInfo& g = plan.groups[gi];
        PSeg sg{};
        sg.h = g.h;
        sg.nblocks = g.nblocks;
        sg.offset = g.offset;
        sg.block0 = g.block0;
        sg.logB = g.logB;
        sg.n = g.n;
        sg.lane = (call != PCALL_SOLVE && c.lane[gi] && persistent_lane_ok(plan, g)) ? 1 : 0;
        sg.tpw = std::max<int>(1, c.tpw[gi]);
        sg.tiles = seg_tiles(g, sg.lane != 0);
        sg.first_item = first;
        first += (sg.tiles + sg.tpw - 1) / sg.tpw;
        segs.push_back(sg);
    }
    c.items = first;
    if (ng == 0) return TP_OK;
    hipError_t e = hipMemcpy(const_cast<PSeg*>(seg_table(plan, call, dt)), segs.data(), ng * sizeof(PSeg),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "persistent segment table upload");
    return TP_OK;
}

tp_status persistent_setup(Plan& plan) {
    const size_t ng = plan.groups.size();
    for (int call = 0; call < 3; ++call)
        for (int dt = 0; dt < 4; ++dt) {
            PersistCfg& c = plan.pcfg[call][dt];
            c = PersistCfg();
            c.lane.resize(ng);
            c.tpw.assign(ng, 1);
            c.order.resize(ng);
            for (size_t i = 0; i < ng; ++i) {
                c.order[i] = static_cast<int32_t>(i);
                // the default body follows the plan's mapping; the single-launch
                // solve runs every degree on wave tiles: one kernel that also
                // held the lane solve's register demand (up to 512 per lane)
                // would run every degree at one wave per SIMD
                c.lane[i] = (call != PCALL_SOLVE && plan.groups[i].n <= kLaneMaxN && plan.mapping != TP_MAP_WAVE);
            }
            c.grid = 1;
        }
    if (ng == 0) return TP_OK;
    hipError_t e = hipMalloc(&plan.segs_dev, 12 * ng * sizeof(PSeg));
    if (e != hipSuccess) return hip_error(e, "persistent segment tables");
    for (int call = 0; call < 3; ++call)
        for (int dt = 0; dt < 4; ++dt) {
            tp_status st = persistent_upload(plan, call, dt);
            if (st != TP_OK) return st;
        }
    return TP_OK;
}

tp_status launch_apply_persistent(const Plan& plan, int op, const void* u, void* v, tp_dtype dt, hipStream_t s) {
    if (plan.groups.empty() || plan.nblocks == 0) return TP_OK;
    switch (dt) {
        case TP_F64: return papply<double, double>(plan, dt, op, u, v, s);
        case TP_F32: return papply<float, float>(plan, dt, op, u, v, s);
        case TP_F16: return papply<_Float16, float>(plan, dt, op, u, v, s);
        case TP_BF16: return papply<bf16_t, float>(plan, dt, op, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_inverse_persistent(const Plan& plan, const void* r, void* x, tp_dtype dt, hipStream_t s) {
    if (plan.groups.empty() || plan.nblocks == 0) return TP_OK;
    switch (dt) {
        case TP_F64: return pinverse<double, double>(plan, dt, r, x, s);
        case TP_F32: return pinverse<float, float>(plan, dt, r, x, s);
        case TP_F16: return pinverse<_Float16, float>(plan, dt, r, x, s);
        case TP_BF16: return pinverse<bf16_t, float>(plan, dt, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_solve_persistent(const Plan& plan, const double* b, double* x, tp_dtype inner, double rtol,
                                  int maxit, int32_t* iters, double* relres, const SolveWork& w, int64_t* nparts,
                                  hipStream_t s) {
    *nparts = 0;
    if (plan.groups.empty() || plan.nblocks == 0) return TP_OK;
    switch (inner) {
        case TP_F64: return psolve<double, RND_NONE>(plan, inner, b, x, rtol, maxit, iters, relres, w, nparts, s);
        case TP_F32: return psolve<float, RND_NONE>(plan, inner, b, x, rtol, maxit, iters, relres, w, nparts, s);
        case TP_F16: return psolve<float, RND_F16>(plan, inner, b, x, rtol, maxit, iters, relres, w, nparts, s);
        case TP_BF16: return psolve<float, RND_BF16>(plan, inner, b, x, rtol, maxit, iters, relres, w, nparts, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported inner precision");
}

}  // namespace tpfdm
