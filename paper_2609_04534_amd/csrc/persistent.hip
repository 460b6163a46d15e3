// Single-launch kernels over all groups of a plan (batches of uneven
// degree).
//
// Every group is a segment of work tiles: 64 blocks per tile for the
// lane-per-block mapping and BPW blocks per tile for the wave-per-tile
// mapping.  The tiles of all segments form one list; apply and
// apply_inverse launch one one-wave workgroup per tile of that list, which
// finds its segment by a scan of the (few) segment starts and runs the
// group's tile body, inlined per degree (no calls, no scratch; each switch
// branch has its own registers).  The solve runs a fixed grid whose
// workgroups walk the list with the grid stride, so its per-workgroup
// summaries fit the plan's partials.  No counters or atomics: the launch is
// capturable in a HIP graph and its results are bitwise those of the
// per-group launches.  Factor tables are loaded per tile.
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
    int64_t tiles_lane;   // tiles of 64 blocks
    int64_t tiles_wave;   // tiles of BPW blocks
    int32_t logB;
    int32_t n;
    int32_t lane;         // apply / apply_inverse use the lane-per-block mapping
    int32_t lane_solve;   // the solve uses the lane-per-block mapping (0 in this launch)
    int64_t first_tile;   // apply / apply_inverse: first tile in the flat tile list
    int64_t first_tile_solve;  // the same for the solve's tiles
};

namespace {

constexpr int kMaxSlab = Slab<8>::BPW * Slab<8>::size;  // largest BPW * slab size over n <= 8

template <int N>
constexpr size_t solve_lds_bytes() {
    return sizeof(SolveLds<N, double>) + 64 * sizeof(double) + 64 * sizeof(double);
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
                                               const TC* __restrict__ ptab, int64_t t0) {
    Pair<N, TC> R;
#pragma unroll
    for (int i = 0; i < N * N; ++i) {
        R.m[i] = ptab[i];
        R.p[i] = ptab[N * N + i];
    }
    const int lb = sg.logB;
    for (int64_t t = t0; t < sg.tiles_lane; t = sg.tiles_lane) {
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
                                               const TC* __restrict__ tab, TC* s1, TC* s2, TC* stab, int64_t t0) {
    using L = Slab<N>;
    ApplyTab<N, TC> A;
    table_to_regs(A.v, tab, stab, ApplyTab<N, TC>::COUNT);
    const GArgs G = seg_args(sg);
    const int lane = threadIdx.x;
    const int lw = lane / L::N2;
    const int lp = lane - lw * L::N2;
    const int li = lp / N, lj = lp - (lp / N) * N;
    const int so = (lw < L::BPW ? lw : 0) * L::size;
    for (int64_t t = t0; t < sg.tiles_wave; t = sg.tiles_wave) {
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
                                          TC* lds, int64_t t0) {
    const int et = sizeof(TC) == 8 ? 0 : 1;
    if constexpr (N <= kLaneMaxN) {
        if (sg.lane) {
            const TC* pt =
                reinterpret_cast<const TC*>(dev_table(tabs, N, op == TP_OP_CELL ? EO_PLAIN_A : EO_PLAIN_K, et));
            if ((static_cast<int64_t>(sizeof(TS)) << sg.logB) >= 128)
                seg_apply_lane<N, TS, TC, true>(u, v, sg, pt, t0);
            else
                seg_apply_lane<N, TS, TC, false>(u, v, sg, pt, t0);
            return;
        }
    }
    const TC* tab = reinterpret_cast<const TC*>(dev_table(tabs, N, op == TP_OP_CELL ? EO_APPLY_A : EO_APPLY_K, et));
    if (vp)
        seg_apply_wave<N, true>(u, v, sg, tab, lds, lds + kMaxSlab, lds + 2 * kMaxSlab, t0);
    else
        seg_apply_wave<N, false>(u, v, sg, tab, lds, lds + kMaxSlab, lds + 2 * kMaxSlab, t0);
}

// ------------------------------------------------------------ inverse
template <int N, typename TS, typename TC, bool NT>
__device__ __forceinline__ void seg_inverse_lane(const TS* __restrict__ r, TS* __restrict__ x, const PSeg& sg,
                                                 const TC* __restrict__ ptab, int64_t t0) {
    Eig<N, TC> E;
#pragma unroll
    for (int i = 0; i < N * N; ++i) E.s[i] = ptab[i];
#pragma unroll
    for (int i = 0; i < N; ++i) E.lam[i] = ptab[N * N + i];
    const int lb = sg.logB;
    for (int64_t t = t0; t < sg.tiles_lane; t = sg.tiles_lane) {
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
                                                 const TC* __restrict__ tab, TC* s1, TC* stab, int64_t t0) {
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
    for (int64_t t = t0; t < sg.tiles_wave; t = sg.tiles_wave) {
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
                                            int64_t t0) {
    const int et = sizeof(TC) == 8 ? 0 : 1;
    if constexpr (N <= kLaneMaxN) {
        if (sg.lane) {
            const TC* pt = reinterpret_cast<const TC*>(dev_table(tabs, N, EO_PLAIN_S, et));
            if ((static_cast<int64_t>(sizeof(TS)) << sg.logB) >= 128)
                seg_inverse_lane<N, TS, TC, true>(r, x, sg, pt, t0);
            else
                seg_inverse_lane<N, TS, TC, false>(r, x, sg, pt, t0);
            return;
        }
    }
    const TC* tab = reinterpret_cast<const TC*>(dev_table(tabs, N, EO_INV, et));
    if (vp)
        seg_inverse_wave<N, true>(r, x, sg, tab, lds, lds + kMaxSlab, t0);
    else
        seg_inverse_wave<N, false>(r, x, sg, tab, lds, lds + kMaxSlab, t0);
}

// ------------------------------------------------------------ solve
template <int N, typename TI, int RND>
__device__ __forceinline__ void seg_solve(const double* b, double* x, const PSeg& sg, const char* tabs, char* lds,
                                          int64_t t0, double rtol, int maxit, int32_t* iters, double* relres,
                                          SolveAcc& acc) {
    using S = EOShape<N>;
    SolveLds<N, TI>& L = *reinterpret_cast<SolveLds<N, TI>*>(lds);
    double* stabA = reinterpret_cast<double*>(lds + sizeof(SolveLds<N, TI>));
    TI* stabS = reinterpret_cast<TI*>(stabA + 64);
    ApplyTab<N, double> A;
    InvTab<N, TI> I;
    table_to_regs(A.v, reinterpret_cast<const double*>(dev_table(tabs, N, EO_APPLY_A, 0)), stabA,
                  ApplyTab<N, double>::COUNT);
    table_to_regs<TI, InvTab<N, TI>::COUNT, false>(
        I.v, reinterpret_cast<const TI*>(dev_table(tabs, N, EO_INV, sizeof(TI) == 8 ? 0 : 1)), stabS,
        S::SE + S::SO + N);
    const TI* lam = stabS + S::SE + S::SO;
    const GArgs G = seg_args(sg);
    for (int64_t t = t0; t < sg.tiles_wave; t = sg.tiles_wave)
        eo_solve_tile<N, TI, RND>(b, x, G, t * Slab<N>::BPW, nvalid_of<N>(G, t), L, A, I, lam, rtol, maxit, iters,
                                  relres, sg.block0, acc);
}


// Segment of the flat tile w: segments in order, each covering the tiles
// [first_tile, first_tile + tiles) of the launch (apply / apply_inverse).
__device__ __forceinline__ int flat_segment(const PSeg* __restrict__ segs, int nseg, int64_t w) {
    int si = 0;
    while (si + 1 < nseg && segs[si + 1].first_tile <= w) ++si;
    return si;
}

// One launch over all groups: one workgroup per tile of the concatenated
// tile list, the group's body inlined per degree (no calls, no scratch).
// Every tile is independent, so the hardware dispatcher balances the mix.
template <typename TS, typename TC>
__global__ __launch_bounds__(64, 2) void k_persist_apply(const TS* __restrict__ u, TS* __restrict__ v,
                                                         const PSeg* __restrict__ segs, int nseg,
                                                         const char* __restrict__ tabs, int op,
                                                         unsigned long long vpmask) {
    __shared__ __align__(16) TC lds[2 * kMaxSlab + 64];
    const int si = flat_segment(segs, nseg, blockIdx.x);
    const PSeg sg = segs[si];
    const int64_t t = static_cast<int64_t>(blockIdx.x) - sg.first_tile;
    const bool vp = si < 64 && ((vpmask >> si) & 1ull);
    switch (sg.n) {
        case 2: seg_apply<2, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
        case 3: seg_apply<3, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
        case 4: seg_apply<4, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
        case 5: seg_apply<5, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
        case 6: seg_apply<6, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
        case 7: seg_apply<7, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
        case 8: seg_apply<8, TS, TC>(u, v, sg, tabs, op, vp, lds, t); break;
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
    const int64_t t = static_cast<int64_t>(blockIdx.x) - sg.first_tile;
    const bool vp = si < 64 && ((vpmask >> si) & 1ull);
    switch (sg.n) {
        case 2: seg_inverse<2, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        case 3: seg_inverse<3, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        case 4: seg_inverse<4, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        case 5: seg_inverse<5, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        case 6: seg_inverse<6, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        case 7: seg_inverse<7, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        case 8: seg_inverse<8, TS, TC>(r, x, sg, tabs, vp, lds, t); break;
        default: break;
    }
}

// The solve over all groups: workgroups walk the concatenated tile list of
// the solve (one tile per step, the group's body inlined per degree).
template <typename TI, int RND>
__global__ __launch_bounds__(64, 2) void k_persist_solve(const double* __restrict__ b, double* __restrict__ x,
                                                         const PSeg* __restrict__ segs, int nseg,
                                                         const char* __restrict__ tabs, double rtol, int maxit,
                                                         int32_t* __restrict__ iters, double* __restrict__ relres,
                                                         int64_t total, SolvePartial* parts) {
    __shared__ __align__(16) char lds[kSolveLdsBytes];
    SolveAcc acc;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int si = 0;
        while (si + 1 < nseg && segs[si + 1].first_tile_solve <= w) ++si;
        const PSeg sg = segs[si];
        const int64_t t = w - sg.first_tile_solve;
        switch (sg.n) {
            case 2: seg_solve<2, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            case 3: seg_solve<3, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            case 4: seg_solve<4, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            case 5: seg_solve<5, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            case 6: seg_solve<6, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            case 7: seg_solve<7, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            case 8: seg_solve<8, TI, RND>(b, x, sg, tabs, lds, t, rtol, maxit, iters, relres, acc); break;
            default: break;
        }
    }
    acc.flush(parts + blockIdx.x);
}

int bpw_of(int n) { return n * n >= 64 ? 1 : 64 / (n * n); }

// Vector pencils per segment (bit i for group i < 64).
unsigned long long vp_mask(const Plan& plan, const void* a, const void* b, int esize) {
    unsigned long long m = 0;
    const int vec = 16 / esize;
    for (size_t i = 0; i < plan.groups.size() && i < 64; ++i) {
        const GroupInfo& g = plan.groups[i];
        if (g.logB != 0 || g.n % vec != 0) continue;
        const uintptr_t pa = reinterpret_cast<uintptr_t>(a) + static_cast<uintptr_t>(g.offset) * esize;
        const uintptr_t pb = reinterpret_cast<uintptr_t>(b) + static_cast<uintptr_t>(g.offset) * esize;
        if (pa % 16 == 0 && pb % 16 == 0) m |= 1ull << i;
    }
    return m;
}

int64_t pgrid(const Plan& plan, const void* kern) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, 0) != hipSuccess || occ <= 0) occ = 8;
    return static_cast<int64_t>(plan.cus) * occ;
}

int64_t total_tiles(const Plan& plan, bool solve) {
    int64_t t = 0;
    for (const auto& g : plan.groups) {
        const bool lane = !solve && g.n <= kLaneMaxN && plan.mapping != TP_MAP_WAVE;  // the solve: wave tiles
        t += lane ? (g.nblocks + 63) / 64 : (g.nblocks + bpw_of(g.n) - 1) / bpw_of(g.n);
    }
    return t;
}

tp_status check_p(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <typename TS, typename TC>
tp_status papply(const Plan& plan, int op, const void* u, void* v, hipStream_t s) {
    const int64_t grid = total_tiles(plan, false);   // one workgroup per tile
    if (grid <= 0) return TP_OK;
    hipLaunchKernelGGL((k_persist_apply<TS, TC>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                       static_cast<const TS*>(u), static_cast<TS*>(v), static_cast<const PSeg*>(plan.segs_dev),
                       static_cast<int>(plan.groups.size()), static_cast<const char*>(plan.eo_dev), op,
                       vp_mask(plan, u, v, sizeof(TS)));
    return check_p("persistent apply launch");
}

template <typename TS, typename TC>
tp_status pinverse(const Plan& plan, const void* r, void* x, hipStream_t s) {
    const int64_t grid = total_tiles(plan, false);
    if (grid <= 0) return TP_OK;
    hipLaunchKernelGGL((k_persist_inverse<TS, TC>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                       static_cast<const TS*>(r), static_cast<TS*>(x), static_cast<const PSeg*>(plan.segs_dev),
                       static_cast<int>(plan.groups.size()), static_cast<const char*>(plan.eo_dev),
                       vp_mask(plan, r, x, sizeof(TS)));
    return check_p("persistent apply_inverse launch");
}

template <typename TI, int RND>
tp_status psolve(const Plan& plan, const double* b, double* x, double rtol, int maxit, int32_t* iters,
                 double* relres, int64_t* nparts, hipStream_t s) {
    const void* kern = reinterpret_cast<const void*>(&k_persist_solve<TI, RND>);
    static int64_t gc = 0;
    if (gc == 0) gc = pgrid(plan, kern);
    const int64_t grid = std::max<int64_t>(1, std::min(gc, total_tiles(plan, true)));
    if (grid > plan.partials_cap) return set_error(TP_ERR_UNSUPPORTED, "too many solve workgroups");
    *nparts = grid;
    hipLaunchKernelGGL((k_persist_solve<TI, RND>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b, x,
                       static_cast<const PSeg*>(plan.segs_dev), static_cast<int>(plan.groups.size()),
                       static_cast<const char*>(plan.eo_dev), rtol, maxit, iters, relres, total_tiles(plan, true),
                       static_cast<SolvePartial*>(plan.partials_dev));
    return check_p("persistent solve launch");
}

}  // namespace

tp_status persistent_setup(Plan& plan) {
    std::vector<PSeg> segs;
    int64_t first = 0, first_solve = 0;
    for (const auto& g : plan.groups) {
        PSeg s{};
        s.h = g.h;
        s.nblocks = g.nblocks;
        s.offset = g.offset;
        s.block0 = g.block0;
        s.tiles_lane = (g.nblocks + 63) / 64;
        s.tiles_wave = (g.nblocks + bpw_of(g.n) - 1) / bpw_of(g.n);
        s.logB = g.logB;
        s.n = g.n;
        s.lane = (g.n <= kLaneMaxN && plan.mapping != TP_MAP_WAVE) ? 1 : 0;
        // the single-launch solve runs every degree on wave tiles: one kernel
        // that also held the lane solve's register demand (up to 512 per
        // lane) would run every degree at one wave per SIMD
        s.lane_solve = 0;
        s.first_tile = first;
        first += s.lane ? s.tiles_lane : s.tiles_wave;
        s.first_tile_solve = first_solve;
        first_solve += s.lane_solve ? s.tiles_lane : s.tiles_wave;
        segs.push_back(s);
    }
    if (segs.empty()) return TP_OK;
    hipError_t e = hipMalloc(&plan.segs_dev, segs.size() * sizeof(PSeg));
    if (e != hipSuccess) return hip_error(e, "persistent segment table");
    e = hipMemcpy(plan.segs_dev, segs.data(), segs.size() * sizeof(PSeg), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "persistent segment table upload");
    return TP_OK;
}

tp_status launch_apply_persistent(const Plan& plan, int op, const void* u, void* v, tp_dtype dt, hipStream_t s) {
    if (plan.groups.empty() || plan.nblocks == 0) return TP_OK;
    switch (dt) {
        case TP_F64: return papply<double, double>(plan, op, u, v, s);
        case TP_F32: return papply<float, float>(plan, op, u, v, s);
        case TP_F16: return papply<_Float16, float>(plan, op, u, v, s);
        case TP_BF16: return papply<bf16_t, float>(plan, op, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_inverse_persistent(const Plan& plan, const void* r, void* x, tp_dtype dt, hipStream_t s) {
    if (plan.groups.empty() || plan.nblocks == 0) return TP_OK;
    switch (dt) {
        case TP_F64: return pinverse<double, double>(plan, r, x, s);
        case TP_F32: return pinverse<float, float>(plan, r, x, s);
        case TP_F16: return pinverse<_Float16, float>(plan, r, x, s);
        case TP_BF16: return pinverse<bf16_t, float>(plan, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_solve_persistent(const Plan& plan, const double* b, double* x, tp_dtype inner, double rtol,
                                  int maxit, int32_t* iters, double* relres, int64_t* nparts, hipStream_t s) {
    *nparts = 0;
    if (plan.groups.empty() || plan.nblocks == 0) return TP_OK;
    switch (inner) {
        case TP_F64: return psolve<double, RND_NONE>(plan, b, x, rtol, maxit, iters, relres, nparts, s);
        case TP_F32: return psolve<float, RND_NONE>(plan, b, x, rtol, maxit, iters, relres, nparts, s);
        case TP_F16: return psolve<float, RND_F16>(plan, b, x, rtol, maxit, iters, relres, nparts, s);
        case TP_BF16: return psolve<float, RND_BF16>(plan, b, x, rtol, maxit, iters, relres, nparts, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported inner precision");
}

}  // namespace tpfdm
