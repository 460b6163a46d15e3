// HIP kernels for gfx950: batched sum-factorized apply, fast-diagonalization
// inverse and block-local iterative-refinement solve.
//
// Two mappings of blocks onto the 64-wide wavefront:
//  * lane-per-block (n <= 4): each lane owns one block; the blocked layout
//    [tile][n][n][n][B] with B >= 64 makes every DoF load/store of a wave one
//    coalesced 64-element transaction (Sec. 2: the cell lane is the fastest
//    address).  All contractions run in registers with the reference matrices
//    as wave-uniform (scalar) operands.
//  * wave-per-block (n >= 5): a workgroup of one wave owns one block; the
//    block's n^3 slab is staged through LDS with coalesced global accesses,
//    and every 1D contraction is a lane-local matrix-vector product on one
//    pencil, with an LDS transpose between axes.
//
// Per-block geometry enters only through three scalars (Sec. 2, Cartesian
// cells stream no geometry): with s_x = h_y h_z / h_x (and cyclic),
//   A u  = s_x (P (x) M (x) M) u + s_y (M (x) P (x) M) u + s_z (M (x) M (x) P) u
//   D^-1 = (S (x) S (x) S) diag(1 / (lam_i s_x + lam_j s_y + lam_k s_z)) (S (x) S (x) S)^T
// where M, P, S, lam are the reference-interval matrices (Sec. 3.1,
// eq. (eval_pipeline); Sec. 5.2, eq. (cell_block)).
#include <algorithm>
#include <type_traits>

#include "lane.h"

namespace tpfdm {

template <int N, typename TS, typename TC, bool NT, int LB>
__global__ __launch_bounds__(64, 2) void k_apply_lane(const TS* __restrict__ u, TS* __restrict__ v, GArgs G,
                                                    Pair<N, TC> R) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G.nblocks) return;
    const int64_t base = G.offset + block_base(g, G.logB, N * N * N);
    const TS* ub = u + base;
    TS* vb = v + base;
    const int lb = LB >= 0 ? LB : G.logB;
    TC sx, sy, sz;
    block_scales(G.h, g, sx, sy, sz);
    TC acc[N * N * N];
    lane_apply<N, TC>([&](int q) { return ldv<NT, TC>(ub + (static_cast<int64_t>(q) << lb)); }, R, sx, sy, sz,
                      acc);
#pragma unroll
    for (int q = 0; q < N * N * N; ++q) stv<NT>(vb + (static_cast<int64_t>(q) << lb), acc[q]);
}

template <int N, typename TS, typename TC, bool NT, int LB>
__global__ __launch_bounds__(64, 3) void k_inverse_lane(const TS* __restrict__ r, TS* __restrict__ x, GArgs G,
                                                      Eig<N, TC> E) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G.nblocks) return;
    const int64_t base = G.offset + block_base(g, G.logB, N * N * N);
    const TS* rb = r + base;
    TS* xb = x + base;
    const int lb = LB >= 0 ? LB : G.logB;
    TC sx, sy, sz;
    block_scales(G.h, g, sx, sy, sz);
    TC v[N * N * N];
#pragma unroll
    for (int q = 0; q < N * N * N; ++q) v[q] = ldv<NT, TC>(rb + (static_cast<int64_t>(q) << lb));
    lane_fdm_inplace<N, TC>(v, E, sx, sy, sz);
#pragma unroll
    for (int q = 0; q < N * N * N; ++q) stv<NT>(xb + (static_cast<int64_t>(q) << lb), v[q]);
}

// Block-local iterative refinement, one block per lane (n <= 4); the body
// is lane_solve_tile (lane.h).  The factor tables come in as kernel
// arguments; M_hat and A_hat are read through their symmetry classes so the
// scalar registers hold each distinct value once (full FP64 tables of both
// operators plus the eigenvectors would not fit).
template <int N, typename TI, int RND, bool NT, int LB>
__global__ __launch_bounds__(64, 1) void k_solve_lane(const double* __restrict__ b, double* __restrict__ x, GArgs G,
                                                      Pair<N, double> PA, Eig<N, TI> E, int64_t ntiles, double rtol,
                                                      int maxit, int32_t* __restrict__ iters,
                                                      double* __restrict__ relres, int64_t block0,
                                                      SolvePartial* __restrict__ parts) {
    const Pair<N, double> RA = sym_pair<N>(PA.m, PA.p);
    __shared__ double xs[N * N * N][64];
    SolveAcc acc;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        lane_solve_tile<N, TI, RND, NT, LB>(b, x, G, RA, E, t, rtol, maxit, iters, relres, block0, acc, xs);
    acc.flush(parts + blockIdx.x);
}

// ============================================================ layout + misc
template <typename E>
__global__ void k_pack(const E* __restrict__ canon, E* __restrict__ blocked, int64_t total, int64_t nblocks,
                       int n3, int logB) {
    const int64_t tileElems = static_cast<int64_t>(n3) << logB;
    const int64_t mask = (int64_t(1) << logB) - 1;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = e / tileElems;
        const int64_t rem = e - t * tileElems;
        const int64_t q = rem >> logB;
        const int64_t blk = (t << logB) + (rem & mask);
        blocked[e] = blk < nblocks ? canon[blk * n3 + q] : E(0);
    }
}

template <typename E>
__global__ void k_unpack(const E* __restrict__ blocked, E* __restrict__ canon, int64_t total, int n3, int logB) {
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < total;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t blk = c / n3;
        const int64_t q = c - blk * n3;
        canon[c] = blocked[block_base(blk, logB, n3) + (q << logB)];
    }
}

// Reduces the per-workgroup partial summaries of one solve into the summary,
// and into host_out (pinned host memory) when that is given, tagged.
__global__ __launch_bounds__(256) void k_summary_reduce(const SolvePartial* __restrict__ parts, int64_t count,
                                                        SolveSummary* __restrict__ out,
                                                        SolveSummary* __restrict__ host_out, int tag) {
    __shared__ int smi[256], snf[256], snn[256];
    __shared__ double smr[256];
    int mi = 0, nf = 0, nn = 0;
    double mr = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) {
        const SolvePartial p = parts[i];
        mi = p.max_iters > mi ? p.max_iters : mi;
        nf += p.n_failed;
        nn += p.nonfinite;
        mr = p.max_relres > mr ? p.max_relres : mr;
    }
    smi[threadIdx.x] = mi;
    snf[threadIdx.x] = nf;
    snn[threadIdx.x] = nn;
    smr[threadIdx.x] = mr;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            smi[threadIdx.x] = smi[threadIdx.x + o] > smi[threadIdx.x] ? smi[threadIdx.x + o] : smi[threadIdx.x];
            snf[threadIdx.x] += snf[threadIdx.x + o];
            snn[threadIdx.x] += snn[threadIdx.x + o];
            smr[threadIdx.x] = smr[threadIdx.x + o] > smr[threadIdx.x] ? smr[threadIdx.x + o] : smr[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        SolveSummary r;
        r.max_iters = smi[0];
        r.n_failed = snf[0];
        r.nonfinite = snn[0];
        r.pad = tag;
        r.max_relres_bits = static_cast<unsigned long long>(__double_as_longlong(smr[0]));
        *out = r;
        if (host_out) *host_out = r;
    }
}

// Pseudo-random fill for scratch vectors (autotuning): splitmix64 of the
// element index and seed, mapped to [-1, 1].
template <typename E>
__global__ void k_fill(E* __restrict__ dst, int64_t n, uint64_t seed, int zero) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * static_cast<uint64_t>(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double v = zero ? 0.0 : static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    stc(dst + i, static_cast<typename std::conditional<sizeof(E) == 8, double, float>::type>(v));
}

// ============================================================ host launchers
namespace {

constexpr int kLaneThreads = 64;   // one wave per workgroup (measured best for n = 4)

template <int N, typename T>
Pair<N, T> make_pair(const double* M, const double* P) {
    Pair<N, T> R;
    for (int i = 0; i < N * N; ++i) {
        R.m[i] = static_cast<T>(M[i]);
        R.p[i] = static_cast<T>(P[i]);
    }
    return R;
}

template <int N, typename T>
Eig<N, T> make_eig(const RefData& ref) {
    Eig<N, T> E;
    for (int i = 0; i < N * N; ++i) E.s[i] = static_cast<T>(ref.S[i]);
    for (int i = 0; i < N; ++i) E.lam[i] = static_cast<T>(ref.lam[i]);
    return E;
}

GArgs gargs(const GroupInfo& g) {
    GArgs a;
    a.h = g.h;
    a.nblocks = g.nblocks;
    a.offset = g.offset;
    a.logB = g.logB;
    return a;
}

tp_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <int N, typename TS, typename TC>
tp_status apply_n(const GroupInfo& g, const double* Mm, const double* Pm, const void* u, void* v, hipStream_t s) {
    const auto R = make_pair<N, TC>(Mm, Pm);
    const unsigned grid = static_cast<unsigned>((g.nblocks + kLaneThreads - 1) / kLaneThreads);
    // B = 64 (the default) is a compile-time layout: every DoF address is
    // the block base plus a constant offset
    if (g.logB == 6)
        hipLaunchKernelGGL((k_apply_lane<N, TS, TC, true, 6>), dim3(grid), dim3(kLaneThreads), 0, s,
                           static_cast<const TS*>(u), static_cast<TS*>(v), gargs(g), R);
    else if (lane_whole_lines<TS>(g.logB))
        hipLaunchKernelGGL((k_apply_lane<N, TS, TC, true, -1>), dim3(grid), dim3(kLaneThreads), 0, s,
                           static_cast<const TS*>(u), static_cast<TS*>(v), gargs(g), R);
    else
        hipLaunchKernelGGL((k_apply_lane<N, TS, TC, false, -1>), dim3(grid), dim3(kLaneThreads), 0, s,
                           static_cast<const TS*>(u), static_cast<TS*>(v), gargs(g), R);
    return check_launch("apply launch");
}

template <int N, typename TS, typename TC>
tp_status inverse_n(const GroupInfo& g, const RefData& ref, const void* r, void* x, hipStream_t s) {
    const auto E = make_eig<N, TC>(ref);
    const unsigned grid = static_cast<unsigned>((g.nblocks + kLaneThreads - 1) / kLaneThreads);
    if (g.logB == 6)
        hipLaunchKernelGGL((k_inverse_lane<N, TS, TC, true, 6>), dim3(grid), dim3(kLaneThreads), 0, s,
                           static_cast<const TS*>(r), static_cast<TS*>(x), gargs(g), E);
    else if (lane_whole_lines<TS>(g.logB))
        hipLaunchKernelGGL((k_inverse_lane<N, TS, TC, true, -1>), dim3(grid), dim3(kLaneThreads), 0, s,
                           static_cast<const TS*>(r), static_cast<TS*>(x), gargs(g), E);
    else
        hipLaunchKernelGGL((k_inverse_lane<N, TS, TC, false, -1>), dim3(grid), dim3(kLaneThreads), 0, s,
                           static_cast<const TS*>(r), static_cast<TS*>(x), gargs(g), E);
    return check_launch("apply_inverse launch");
}

template <typename TS, typename TC>
tp_status apply_dispatch(const GroupInfo& g, const double* Mm, const double* Pm, const void* u, void* v,
                         hipStream_t s) {
    switch (g.n) {
        case 2: return apply_n<2, TS, TC>(g, Mm, Pm, u, v, s);
        case 3: return apply_n<3, TS, TC>(g, Mm, Pm, u, v, s);
        case 4: return apply_n<4, TS, TC>(g, Mm, Pm, u, v, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

template <typename TS, typename TC>
tp_status inverse_dispatch(const GroupInfo& g, const RefData& ref, const void* r, void* x, hipStream_t s) {
    switch (g.n) {
        case 2: return inverse_n<2, TS, TC>(g, ref, r, x, s);
        case 3: return inverse_n<3, TS, TC>(g, ref, r, x, s);
        case 4: return inverse_n<4, TS, TC>(g, ref, r, x, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}


template <int N, typename TI, int RND>
tp_status solve_lane_n(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                       int32_t* iters, double* relres, const SolveWork& w, int64_t part_base, int64_t* nparts,
                       hipStream_t s) {
    const RefData& ref = plan.ref[N];
    const auto PA = make_pair<N, double>(ref.M, ref.A);
    const auto E = make_eig<N, TI>(ref);
    const int64_t ntiles = (g.nblocks + 63) / 64;
    const bool nt = lane_whole_lines<double>(g.logB);
    const void* kern = g.logB == 6 ? reinterpret_cast<const void*>(&k_solve_lane<N, TI, RND, true, 6>)
                       : nt        ? reinterpret_cast<const void*>(&k_solve_lane<N, TI, RND, true, -1>)
                                   : reinterpret_cast<const void*>(&k_solve_lane<N, TI, RND, false, -1>);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, 0) != hipSuccess || occ <= 0) occ = 1;
    occ = std::min(occ, kMaxWgPerCu);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ntiles, static_cast<int64_t>(plan.cus) * occ));
    if (part_base + grid > w.cap) return set_error(TP_ERR_UNSUPPORTED, "too many solve workgroups");
    SolvePartial* parts = w.parts + part_base;
    const int64_t block0 = g.block0;
    if (g.logB == 6)
        hipLaunchKernelGGL((k_solve_lane<N, TI, RND, true, 6>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b,
                           x, gargs(g), PA, E, ntiles, rtol, maxit, iters, relres, block0, parts);
    else if (nt)
        hipLaunchKernelGGL((k_solve_lane<N, TI, RND, true, -1>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b,
                           x, gargs(g), PA, E, ntiles, rtol, maxit, iters, relres, block0, parts);
    else
        hipLaunchKernelGGL((k_solve_lane<N, TI, RND, false, -1>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                           b, x, gargs(g), PA, E, ntiles, rtol, maxit, iters, relres, block0, parts);
    *nparts = grid;
    return check_launch("solve (lane) launch");
}

template <typename TI, int RND>
tp_status solve_lane_dispatch(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                              int32_t* iters, double* relres, const SolveWork& w, int64_t part_base, int64_t* nparts,
                       hipStream_t s) {
    switch (g.n) {
        case 2: return solve_lane_n<2, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case 3: return solve_lane_n<3, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case 4: return solve_lane_n<4, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}
}  // namespace

tp_status launch_apply(const Plan& plan, const GroupInfo& g, const double* Pm, const void* u, void* v,
                       tp_dtype dt, hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    const double* Mm = plan.ref[g.n].M;
    switch (dt) {
        case TP_F64: return apply_dispatch<double, double>(g, Mm, Pm, u, v, s);
        case TP_F32: return apply_dispatch<float, float>(g, Mm, Pm, u, v, s);
        case TP_F16: return apply_dispatch<_Float16, float>(g, Mm, Pm, u, v, s);
        case TP_BF16: return apply_dispatch<bf16_t, float>(g, Mm, Pm, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_inverse(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                         hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    const RefData& ref = plan.ref[g.n];
    switch (dt) {
        case TP_F64: return inverse_dispatch<double, double>(g, ref, r, x, s);
        case TP_F32: return inverse_dispatch<float, float>(g, ref, r, x, s);
        case TP_F16: return inverse_dispatch<_Float16, float>(g, ref, r, x, s);
        case TP_BF16: return inverse_dispatch<bf16_t, float>(g, ref, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_solve_lane(const Plan& plan, const GroupInfo& g, const double* b, double* x, tp_dtype inner,
                            double rtol, int maxit, int32_t* iters, double* relres, const SolveWork& w,
                            int64_t part_base, int64_t* nparts, hipStream_t s) {
    *nparts = 0;
    if (g.nblocks == 0) return TP_OK;
    switch (inner) {
        case TP_F64:
            return solve_lane_dispatch<double, RND_NONE>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_F32:
            return solve_lane_dispatch<float, RND_NONE>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_F16:
            return solve_lane_dispatch<float, RND_F16>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_BF16:
            return solve_lane_dispatch<float, RND_BF16>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported inner precision");
}

tp_status launch_fill(void* dst, int64_t n, tp_dtype dt, uint64_t seed, bool zero, hipStream_t s) {
    if (n <= 0) return TP_OK;
    const unsigned grid = static_cast<unsigned>((n + 255) / 256);
    switch (dt) {
        case TP_F64:
            hipLaunchKernelGGL((k_fill<double>), dim3(grid), dim3(256), 0, s, static_cast<double*>(dst), n, seed, zero);
            break;
        case TP_F32:
            hipLaunchKernelGGL((k_fill<float>), dim3(grid), dim3(256), 0, s, static_cast<float*>(dst), n, seed, zero);
            break;
        case TP_F16:
            hipLaunchKernelGGL((k_fill<_Float16>), dim3(grid), dim3(256), 0, s, static_cast<_Float16*>(dst), n, seed,
                               zero);
            break;
        case TP_BF16:
            hipLaunchKernelGGL((k_fill<bf16_t>), dim3(grid), dim3(256), 0, s, static_cast<bf16_t*>(dst), n, seed, zero);
            break;
    }
    return check_launch("fill launch");
}

tp_status launch_pack(const GroupInfo& g, const void* src, void* dst, int esize, bool to_blocked,
                      hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    const int n3 = g.n * g.n * g.n;
    const int64_t tiles = (g.nblocks + (int64_t(1) << g.logB) - 1) >> g.logB;
    const int64_t total = to_blocked ? ((tiles * n3) << g.logB) : g.nblocks * n3;
    const int threads = 256;
    int64_t blocks = (total + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
#define TP_PACK_CASE(T)                                                                                        \
    if (to_blocked)                                                                                            \
        hipLaunchKernelGGL((k_pack<T>), dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, s,              \
                           static_cast<const T*>(src) + g.canon, static_cast<T*>(dst) + g.offset, total,      \
                           g.nblocks, n3, g.logB);                                                             \
    else                                                                                                       \
        hipLaunchKernelGGL((k_unpack<T>), dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, s,            \
                           static_cast<const T*>(src) + g.offset, static_cast<T*>(dst) + g.canon, total,      \
                           n3, g.logB);
    switch (esize) {
        case 2: { TP_PACK_CASE(uint16_t) break; }
        case 4: { TP_PACK_CASE(uint32_t) break; }
        case 8: { TP_PACK_CASE(uint64_t) break; }
        default: return set_error(TP_ERR_UNSUPPORTED, "element size");
    }
#undef TP_PACK_CASE
    return check_launch("pack launch");
}

tp_status launch_summary_reduce(const SolveWork& w, int64_t nparts, SolveSummary* host_out, int tag, hipStream_t s) {
    hipLaunchKernelGGL(k_summary_reduce, dim3(1), dim3(256), 0, s, static_cast<const SolvePartial*>(w.parts), nparts,
                       w.summary, host_out, tag);
    return check_launch("solve summary reduction");
}

}  // namespace tpfdm
