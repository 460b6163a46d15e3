// The coupled SIPG operator on a uniform Cartesian box mesh: one fused
// kernel computes v = A u with A = A^vol + A^face (Sec. 3, eq. (sipg),
// eq. (operator_split)), homogeneous Dirichlet data imposed by Nitsche's
// terms on the boundary faces.
//
// Row of cell c.  The cell-diagonal block is the Kronecker sum of the cell
// block (eq. (cell_block), A_hat = K_hat + the own-side blocks of both
// interior face stencils) plus, on a boundary face, the difference between
// the Nitsche own-side block and the interior one.  The off-diagonal blocks
// couple c to its face neighbours through N^{-+} and N^{+-} of
// eq. (face_factorized) in the normal slot and the mass matrix in the two
// tangential slots.  With e0, e1 the endpoint values (unit vectors of the
// Gauss-Lobatto basis) and g0, g1 the reference endpoint derivatives, every
// face term is rank two in the normal slot (the rank-two flux structure of
// Sec. 6.3):
//
//   (N w)_i = e_end,i alpha(w) + g_end,i beta(w),    then (x) M (x) M,
//
// where, for the face at the cell's upper end along an axis (normal slot
// index k, source block w):
//   interior:  w = upper neighbour, alpha = -sigma w_0 - 1/2 g0.w,  beta = +1/2 w_0
//   boundary:  w = the cell itself, alpha = -1/2 g1.w,              beta = -1/2 w_{n-1}
// and for the lower end:
//   interior:  w = lower neighbour, alpha = -sigma w_{n-1} + 1/2 g1.w, beta = -1/2 w_{n-1}
//   boundary:  w = the cell itself, alpha = +1/2 g0.w,                 beta = +1/2 w_0
// (sigma = C p (p+1), Sec. 6.2; every term scales with s_d = h_o1 h_o2 / h_d
// like the volume term of that axis).  The face-only operator A^face uses
// A_hat - K_hat for the cell-diagonal Kronecker sum.
//
// Unlike the paper's separate face-exchange sweeps, which read and update
// the output's face layers once per axis, the kernel is cell-centric: every
// cell reads its six neighbours (from cache: the same blocks are its
// neighbours' own inputs) and writes its output block once, so HBM sees one
// read of u and one write of v.  Each interior face is evaluated from both
// sides, which costs arithmetic, not HBM bytes.
//
// Mesh order: cell (cx, cy, cz) is block c = (cx m_y + cy) m_z + cz of the
// blocked layout, so the B cells of a tile are consecutive along z.
#include <algorithm>

#include "lane.h"

namespace tpfdm {

struct MeshArgs {
    int64_t ncells;
    int64_t offset;
    int logB;
    int mx, my, mz;
    double sx, sy, sz;   // s_d = h_o1 h_o2 / h_d
};

template <int N, typename T>
struct FaceRef {        // reference endpoint derivatives and penalty C p (p+1)
    T g0[N];
    T g1[N];
    T sigma;
};

namespace {

// DoF index of (normal layer k, tangential a, b) for a face normal to axis D
// (a, b are the two other axes in increasing order).
template <int N, int D>
__device__ __forceinline__ constexpr int fq(int k, int a, int b) {
    return D == 0 ? (k * N + a) * N + b : D == 1 ? (a * N + k) * N + b : (a * N + b) * N + k;
}

// Adds one face's term to the lane's output block acc.  w: the source
// block's DoF 0 (neighbour or the cell itself, see the header), s: s_D.
// Each n x n slab (beta: one layer of the source; alpha: a weighted sum of
// its layers) gets the tangential mass contraction M (.) M in two passes:
// rows are loaded, contracted along the second tangential index and parked
// in the lane's LDS slab sb[e][lane]; columns are read back, contracted
// along the first and accumulated into acc.  Only one row of loads is live
// next to acc, which keeps the n = 4 FP64 block (128 VGPRs) spill-free.
template <int N, int D, bool UP, typename TS, typename TC, int LB>
__device__ __forceinline__ void lane_face(const TS* __restrict__ w, int lb, bool interior, const TC* M,
                                          const FaceRef<N, TC>& F, TC s, TC (&acc)[N * N * N], TC (*sb)[64]) {
    constexpr int KS = D == 0 ? N * N : D == 1 ? N : 1;   // DoF stride of the normal index
    constexpr int kend = UP ? N - 1 : 0;
    const int l = LB >= 0 ? LB : lb;
    const int lane = threadIdx.x;
    auto ld = [&](const TS* p, int q) { return ldc<TC>(p + (static_cast<int64_t>(q) << l)); };
    // row a of a slab (already weighted) -> sb[a][.] = M-contracted row
    auto park_row = [&](int a, const TC (&r)[N]) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
            TC t = TC(0);
#pragma unroll
            for (int bb = 0; bb < N; ++bb) t = fma(M[b * N + bb], r[bb], t);
            sb[a * N + b][lane] = t;
        }
    };
    // column b of the parked slab, contracted along a
    auto column = [&](int b, TC (&out)[N]) {
        TC col[N];
#pragma unroll
        for (int a = 0; a < N; ++a) col[a] = sb[a * N + b][lane];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            TC t = TC(0);
#pragma unroll
            for (int aa = 0; aa < N; ++aa) t = fma(M[a * N + aa], col[aa], t);
            out[a] = t;
        }
    };
    // beta slab: the source's layer 0 or n-1, weighted +-1/2, spread over
    // all layers of acc with the endpoint derivative g_end
    const bool first = (UP == interior);
    const TC cb = first ? TC(0.5) * s : TC(-0.5) * s;
    const TS* wl = w + (static_cast<int64_t>(first ? 0 : (N - 1) * KS) << l);
#pragma unroll
    for (int a = 0; a < N; ++a) {
        __builtin_amdgcn_sched_barrier(0);
        TC r[N];
#pragma unroll
        for (int b = 0; b < N; ++b) r[b] = cb * ld(wl, fq<N, D>(0, a, b));
        park_row(a, r);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
        TC bt[N];
        column(b, bt);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const TC gk = UP ? F.g1[k] : F.g0[k];
#pragma unroll
            for (int a = 0; a < N; ++a) acc[fq<N, D>(k, a, b)] = fma(gk, bt[a], acc[fq<N, D>(k, a, b)]);
        }
    }
    // alpha slab: sum_k ca_k w_k over the normal layers, into layer kend
    TC ca[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const TC in = UP ? fma(TC(-0.5), F.g0[k], k == 0 ? -F.sigma : TC(0))
                         : fma(TC(0.5), F.g1[k], k == N - 1 ? -F.sigma : TC(0));
        const TC bd = UP ? TC(-0.5) * F.g1[k] : TC(0.5) * F.g0[k];
        ca[k] = s * (interior ? in : bd);
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        __builtin_amdgcn_sched_barrier(0);
        TC r[N];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            TC t = TC(0);
#pragma unroll
            for (int k = 0; k < N; ++k) t = fma(ca[k], ld(w, fq<N, D>(k, a, b)), t);
            r[b] = t;
        }
        park_row(a, r);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
        TC at[N];
        column(b, at);
#pragma unroll
        for (int a = 0; a < N; ++a) acc[fq<N, D>(kend, a, b)] += at[a];
    }
}

// One cell per lane (n <= 4).  The cell's own block is read with cached
// loads (it is also a face source of its neighbours); v is streamed out.
template <int N, typename TS, typename TC, bool NT, int LB>
__global__ __launch_bounds__(64, 2) void k_sipg_lane(const TS* __restrict__ u, TS* __restrict__ v, MeshArgs G,
                                                   Pair<N, TC> R, FaceRef<N, TC> F) {
    constexpr int N3 = N * N * N;
    __shared__ TC sb[N * N][64];
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (c >= G.ncells) return;
    const int lb = LB >= 0 ? LB : G.logB;
    const uint32_t cu = static_cast<uint32_t>(c);
    const uint32_t cz = cu % static_cast<uint32_t>(G.mz);
    const uint32_t rr = cu / static_cast<uint32_t>(G.mz);
    const uint32_t cy = rr % static_cast<uint32_t>(G.my);
    const uint32_t cx = rr / static_cast<uint32_t>(G.my);
    const TS* ub = u + G.offset;
    const TS* own = ub + block_base(c, lb, N3);
    const TC sx = static_cast<TC>(G.sx), sy = static_cast<TC>(G.sy), sz = static_cast<TC>(G.sz);
    // face terms first, then the cell-diagonal Kronecker sum accumulated on
    // top: no face state is live while the volume product holds its planes
    TC acc[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) acc[q] = TC(0);
    const int64_t syz = static_cast<int64_t>(G.my) * G.mz;
    // the source cell of a face: the neighbour, or the cell itself on the
    // boundary (an index select, so the kernel stays one basic block)
    auto src = [&](bool interior, int64_t d) { return ub + block_base(interior ? c + d : c, lb, N3); };
    {
        const bool lo = cx > 0, hi = cx + 1 < static_cast<uint32_t>(G.mx);
        lane_face<N, 0, false, TS, TC, LB>(src(lo, -syz), lb, lo, R.m, F, sx, acc, sb);
        lane_face<N, 0, true, TS, TC, LB>(src(hi, syz), lb, hi, R.m, F, sx, acc, sb);
    }
    {
        const bool lo = cy > 0, hi = cy + 1 < static_cast<uint32_t>(G.my);
        lane_face<N, 1, false, TS, TC, LB>(src(lo, -G.mz), lb, lo, R.m, F, sy, acc, sb);
        lane_face<N, 1, true, TS, TC, LB>(src(hi, G.mz), lb, hi, R.m, F, sy, acc, sb);
    }
    {
        const bool lo = cz > 0, hi = cz + 1 < static_cast<uint32_t>(G.mz);
        lane_face<N, 2, false, TS, TC, LB>(src(lo, -1), lb, lo, R.m, F, sz, acc, sb);
        lane_face<N, 2, true, TS, TC, LB>(src(hi, 1), lb, hi, R.m, F, sz, acc, sb);
    }
    __builtin_amdgcn_sched_barrier(0);
    lane_apply<N, TC, false, true>([&](int q) { return ldc<TC>(own + (static_cast<int64_t>(q) << lb)); }, R, sx, sy,
                                   sz, acc);
    TS* vb = v + G.offset + block_base(c, lb, N3);
#pragma unroll
    for (int q = 0; q < N3; ++q) stv<NT>(vb + (static_cast<int64_t>(q) << lb), acc[q]);
}

tp_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <int N, typename TC>
void sipg_tables(const Plan& plan, bool face_only, Pair<N, TC>& R, FaceRef<N, TC>& F) {
    const RefData& ref = plan.ref[N];
    for (int i = 0; i < N * N; ++i) {
        R.m[i] = static_cast<TC>(ref.M[i]);
        R.p[i] = static_cast<TC>(face_only ? ref.A[i] - ref.K[i] : ref.A[i]);
    }
    double g0[N], g1[N];
    endpoint_derivatives(N, g0, g1);
    for (int i = 0; i < N; ++i) {
        F.g0[i] = static_cast<TC>(g0[i]);
        F.g1[i] = static_cast<TC>(g1[i]);
    }
    F.sigma = static_cast<TC>(plan.penalty_C * (N - 1) * N);
}

template <int N, typename TS, typename TC>
tp_status sipg_lane_n(const Plan& plan, const MeshArgs& G, bool face_only, const void* u, void* v, hipStream_t s) {
    Pair<N, TC> R;
    FaceRef<N, TC> F;
    sipg_tables<N, TC>(plan, face_only, R, F);
    const unsigned grid = static_cast<unsigned>((G.ncells + 63) / 64);
    const TS* ui = static_cast<const TS*>(u);
    TS* vo = static_cast<TS*>(v);
    if (G.logB == 6)
        hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, true, 6>), dim3(grid), dim3(64), 0, s, ui, vo, G, R, F);
    else if (lane_whole_lines<TS>(G.logB))
        hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, true, -1>), dim3(grid), dim3(64), 0, s, ui, vo, G, R, F);
    else
        hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, false, -1>), dim3(grid), dim3(64), 0, s, ui, vo, G, R, F);
    return check_launch("SIPG apply launch");
}

template <typename TS, typename TC>
tp_status sipg_dispatch(const Plan& plan, const MeshArgs& G, int n, bool face_only, const void* u, void* v,
                        hipStream_t s) {
    switch (n) {
        case 2: return sipg_lane_n<2, TS, TC>(plan, G, face_only, u, v, s);
        case 3: return sipg_lane_n<3, TS, TC>(plan, G, face_only, u, v, s);
        case 4: return sipg_lane_n<4, TS, TC>(plan, G, face_only, u, v, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "the SIPG operator supports n <= 4");
}

}  // namespace

tp_status launch_sipg(const Plan& plan, const GroupInfo& g, bool face_only, const void* u, void* v, tp_dtype dt,
                      hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    MeshArgs G;
    G.ncells = g.nblocks;
    G.offset = g.offset;
    G.logB = g.logB;
    G.mx = plan.mesh_m[0];
    G.my = plan.mesh_m[1];
    G.mz = plan.mesh_m[2];
    const double hx = plan.mesh_h[0], hy = plan.mesh_h[1], hz = plan.mesh_h[2];
    G.sx = hy * hz / hx;
    G.sy = hx * hz / hy;
    G.sz = hx * hy / hz;
    switch (dt) {
        case TP_F64: return sipg_dispatch<double, double>(plan, G, g.n, face_only, u, v, s);
        case TP_F32: return sipg_dispatch<float, float>(plan, G, g.n, face_only, u, v, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "the SIPG operator supports TP_F64 and TP_F32");
}

}  // namespace tpfdm
