// Device code of the coupled SIPG operator on a uniform Cartesian box mesh
// (shared by sipg.hip and pcg.hip).  One fused kernel computes v = A u with A = A^vol + A^face (Sec. 3, eq. (sipg),
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
#pragma once

#include "eo.h"
#include "lane.h"

namespace tpfdm {

// Device-side state of a PCG solve (pcg.hip; the multigrid kernels of a
// solve read its done flag).  done: 0 running, 1 converged, 2 breakdown or
// a non-finite scalar, 3 iteration limit.
struct PcgState {
    double rz, pq, rr, bb, alpha, beta, tol2;
    int iter, done, maxit;
    int norm;   // stopping test on 0: (r, r), 1: (r, z) (tol2 scaled to match)
};

// Sum of a double over the 64 lanes of a wave.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

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

// DoF index of (normal layer k, tangential a, b) for a face normal to axis D
// (a, b are the two other axes in increasing order).
template <int N, int D>
__device__ __forceinline__ constexpr int fq(int k, int a, int b) {
    return D == 0 ? (k * N + a) * N + b : D == 1 ? (a * N + k) * N + b : (a * N + b) * N + k;
}

// Forces the values to be computed here: the compiler would otherwise sink
// arithmetic below later loads (past scheduling barriers), keeping all the
// loaded layers live at once.
template <typename T, int K>
__device__ __forceinline__ void pin(T (&a)[K]) {
#pragma unroll
    for (int e = 0; e < K; ++e) asm volatile("" : "+v"(a[e]));
}

// Adds one face's term to the lane's output block acc.  w: the source
// block's DoF 0 (neighbour or the cell itself, see the header), s: s_D.
// The source's n layers (normal index) are loaded once, layer by layer:
// alpha = sum_k ca_k w_k accumulates in registers, and the beta slab (the
// source's layer 0 or n-1, weighted +-1/2) is taken from the same loads.
// Each slab gets the tangential mass contraction M (.) M in two passes:
// rows are contracted along the second tangential index and parked in the
// lane's LDS slabs (sa: alpha, sbt: beta; [e][lane], private to the lane);
// columns are read back, contracted along the first and accumulated into
// acc (alpha into layer kend, beta into every layer with weight g_end).
template <int N, int D, bool UP, typename TS, typename TC, int LB>
__device__ __forceinline__ void lane_face(const TS* __restrict__ w, int lb, bool interior, const TC* M,
                                          const FaceRef<N, TC>& F, TC s, TC (&acc)[N * N * N], TC (*sa)[64],
                                          TC (*sbt)[64]) {
    constexpr int kend = UP ? N - 1 : 0;
    const int l = LB >= 0 ? LB : lb;
    const int lane = threadIdx.x;
    auto ld = [&](int q) { return ldc<TC>(w + (static_cast<int64_t>(q) << l)); };
    // row r (already weighted) -> dst[a][.] = M-contracted row (+ dst when ADD)
    auto park_row = [&](TC(*dst)[64], int a, const TC* r, bool add) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
            TC t = add ? dst[a * N + b][lane] : TC(0);
#pragma unroll
            for (int bb = 0; bb < N; ++bb) t = fma(M[b * N + bb], r[bb], t);
            dst[a * N + b][lane] = t;
        }
    };
    // column b of a parked slab, contracted along a
    auto column = [&](TC(*src)[64], int b, TC (&out)[N]) {
        TC col[N];
#pragma unroll
        for (int a = 0; a < N; ++a) col[a] = src[a * N + b][lane];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            TC t = TC(0);
#pragma unroll
            for (int aa = 0; aa < N; ++aa) t = fma(M[a * N + aa], col[aa], t);
            out[a] = t;
        }
    };
    // beta comes from layer 0 when the face is interior at the upper end or
    // boundary at the lower end, else from layer n-1
    const bool first = (UP == interior);
    const TC cb0 = first ? TC(0.5) * s : TC(0);    // weight of layer 0
    const TC cbn = first ? TC(0) : TC(-0.5) * s;   // weight of layer n-1
    TC ca[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const TC in = UP ? fma(TC(-0.5), F.g0[k], k == 0 ? -F.sigma : TC(0))
                         : fma(TC(0.5), F.g1[k], k == N - 1 ? -F.sigma : TC(0));
        const TC bd = UP ? TC(-0.5) * F.g1[k] : TC(0.5) * F.g0[k];
        ca[k] = s * (interior ? in : bd);
    }
    {
        // the next layer's loads in flight while one is accumulated, except
        // where the lane's output block already fills half the register file
        // (n = 4 in FP64)
        constexpr bool DB = N * N * N * sizeof(TC) < 512;
        TC sl[N][N], lay[DB ? 2 : 1][N * N];
        auto load_layer = [&](int k, TC(&dst)[N * N]) {
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int b = 0; b < N; ++b) dst[a * N + b] = ld(fq<N, D>(k, a, b));
        };
        __builtin_amdgcn_sched_barrier(0);
        load_layer(0, lay[0]);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (DB) {
                if (k + 1 < N) load_layer(k + 1, lay[(k + 1) & 1]);
            } else if (k > 0) {
                load_layer(k, lay[0]);
            }
            TC* cur = lay[DB ? (k & 1) : 0];
#pragma unroll
            for (int a = 0; a < N; ++a) {
#pragma unroll
                for (int b = 0; b < N; ++b)
                    sl[a][b] = k == 0 ? ca[0] * cur[a * N + b] : fma(ca[k], cur[a * N + b], sl[a][b]);
                pin(sl[a]);
            }
            if (k == 0 || k == N - 1) {
                // beta = cb0 w_0 + cbn w_{n-1}: one of the two weights is zero
                // per lane, so the slab needs no per-lane branch
                const TC cw = k == 0 ? cb0 : cbn;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    TC r[N];
#pragma unroll
                    for (int b = 0; b < N; ++b) r[b] = cw * cur[a * N + b];
                    park_row(sbt, a, r, k != 0);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < N; ++a) park_row(sa, a, sl[a], false);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
        TC at[N], bt[N];
        column(sa, b, at);
        column(sbt, b, bt);
#pragma unroll
        for (int a = 0; a < N; ++a) acc[fq<N, D>(kend, a, b)] += at[a];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const TC gk = UP ? F.g1[k] : F.g0[k];
#pragma unroll
            for (int a = 0; a < N; ++a) acc[fq<N, D>(k, a, b)] = fma(gk, bt[a], acc[fq<N, D>(k, a, b)]);
        }
    }
}

// The face term in the Hermite-type basis (eq. (hermite_traces_3d)): the
// trace and the normal derivative of a cell at a face are its two layers
// next to that face, so alpha and beta read two layers of the source (the
// neighbour's layers next to the face, or on a boundary face the cell's
// own), and the result lands in the cell's two layers next to the face:
// alpha in the trace layer kend, beta in the derivative layer next to it.
// Same weights as lane_face (only the endpoint derivative of the
// derivative layer is nonzero in this basis), same two-pass tangential mass.
template <int N, int D, bool UP, typename TS, typename TC, int LB>
__device__ __forceinline__ void lane_face_h(const TS* __restrict__ w, int lb, bool interior, const TC* M,
                                            const FaceRef<N, TC>& F, TC s, TC (&acc)[N * N * N], TC (*sa)[64],
                                            TC (*sbt)[64]) {
    static_assert(N >= 4, "the Hermite-type basis has n >= 4");
    constexpr int kend = UP ? N - 1 : 0;
    constexpr int kder = UP ? N - 2 : 1;
    constexpr int LS = D == 0 ? N * N : D == 1 ? N : 1;   // stride of the normal index
    const int l = LB >= 0 ? LB : lb;
    const int lane = threadIdx.x;
    // source layers k0, k0 + 1: 0, 1 when the face is interior at the upper
    // end or boundary at the lower end, else n-2, n-1
    const bool first = (UP == interior);
    const TS* wk = w + (static_cast<int64_t>(first ? 0 : (N - 2) * LS) << l);
    auto ld = [&](int q) { return ldc<TC>(wk + (static_cast<int64_t>(q) << l)); };
    auto park_row = [&](TC(*dst)[64], int a, const TC* r, bool add) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
            TC t = add ? dst[a * N + b][lane] : TC(0);
#pragma unroll
            for (int bb = 0; bb < N; ++bb) t = fma(M[b * N + bb], r[bb], t);
            dst[a * N + b][lane] = t;
        }
    };
    auto column = [&](TC(*src)[64], int b, TC (&out)[N]) {
        TC col[N];
#pragma unroll
        for (int a = 0; a < N; ++a) col[a] = src[a * N + b][lane];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            TC t = TC(0);
#pragma unroll
            for (int aa = 0; aa < N; ++aa) t = fma(M[a * N + aa], col[aa], t);
            out[a] = t;
        }
    };
    // alpha weights of all n layers (as in lane_face), then those of the two
    // source layers selected per lane
    TC ca[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const TC in = UP ? fma(TC(-0.5), F.g0[k], k == 0 ? -F.sigma : TC(0))
                         : fma(TC(0.5), F.g1[k], k == N - 1 ? -F.sigma : TC(0));
        const TC bd = UP ? TC(-0.5) * F.g1[k] : TC(0.5) * F.g0[k];
        ca[k] = s * (interior ? in : bd);
    }
    const TC c0 = first ? ca[0] : ca[N - 2], c1 = first ? ca[1] : ca[N - 1];
    const TC d0 = first ? TC(0.5) * s : TC(0), d1 = first ? TC(0) : TC(-0.5) * s;
    {
        TC sl[N][N], lay[N * N];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int b = 0; b < N; ++b) lay[a * N + b] = ld(fq<N, D>(t, a, b));
            const TC ct = t == 0 ? c0 : c1;
#pragma unroll
            for (int a = 0; a < N; ++a) {
#pragma unroll
                for (int b = 0; b < N; ++b) sl[a][b] = t == 0 ? ct * lay[a * N + b] : fma(ct, lay[a * N + b], sl[a][b]);
                pin(sl[a]);
            }
            // beta = d0 w_k0 + d1 w_k0+1: one weight is zero per lane
            const TC dt = t == 0 ? d0 : d1;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                TC r[N];
#pragma unroll
                for (int b = 0; b < N; ++b) r[b] = dt * lay[a * N + b];
                park_row(sbt, a, r, t != 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < N; ++a) park_row(sa, a, sl[a], false);
    }
    __builtin_amdgcn_sched_barrier(0);
    const TC gk = UP ? F.g1[kder] : F.g0[kder];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        TC at[N], bt[N];
        column(sa, b, at);
        column(sbt, b, bt);
#pragma unroll
        for (int a = 0; a < N; ++a) {
            acc[fq<N, D>(kend, a, b)] += at[a];
            acc[fq<N, D>(kder, a, b)] = fma(gk, bt[a], acc[fq<N, D>(kder, a, b)]);
        }
    }
}

// (A u) of cell c into acc (the row of eq. (sipg) for one cell, see the
// header): the six face terms first, then the cell-diagonal Kronecker sum
// accumulated on top, so no face state is live while the volume product
// holds its planes.  sa, sbt: the lane's LDS slabs (N^2 x 64 each).
template <int N, typename TS, typename TC, int LB, bool HERM = false>
__device__ __forceinline__ void sipg_cell(const TS* __restrict__ u, const MeshArgs& G, const Pair<N, TC>& R,
                                          const FaceRef<N, TC>& F, int64_t c, TC (&acc)[N * N * N],
                                          TC (*sa)[64], TC (*sbt)[64]) {
    constexpr int N3 = N * N * N;
    const int lb = LB >= 0 ? LB : G.logB;
    const uint32_t cu = static_cast<uint32_t>(c);
    const uint32_t cz = cu % static_cast<uint32_t>(G.mz);
    const uint32_t rr = cu / static_cast<uint32_t>(G.mz);
    const uint32_t cy = rr % static_cast<uint32_t>(G.my);
    const uint32_t cx = rr / static_cast<uint32_t>(G.my);
    const TS* ub = u + G.offset;
    const TS* own = ub + block_base(c, lb, N3);
    const TC sx = static_cast<TC>(G.sx), sy = static_cast<TC>(G.sy), sz = static_cast<TC>(G.sz);
#pragma unroll
    for (int q = 0; q < N3; ++q) acc[q] = TC(0);
    const int64_t syz = static_cast<int64_t>(G.my) * G.mz;
    // the source cell of a face: the neighbour, or the cell itself on the
    // boundary (an index select, so the kernel stays one basic block)
    auto src = [&](bool interior, int64_t d) { return ub + block_base(interior ? c + d : c, lb, N3); };
    // the face routine of the basis: Hermite-type (two layers) or Lagrange
    auto face = [&](auto Dc, auto UPc, const TS* w, bool interior, TC sd) {
        constexpr int D = decltype(Dc)::value;
        constexpr bool UP = decltype(UPc)::value;
        if constexpr (HERM)
            lane_face_h<N, D, UP, TS, TC, LB>(w, lb, interior, R.m, F, sd, acc, sa, sbt);
        else
            lane_face<N, D, UP, TS, TC, LB>(w, lb, interior, R.m, F, sd, acc, sa, sbt);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using BF = std::integral_constant<bool, false>;
    using BT = std::integral_constant<bool, true>;
    {
        const bool lo = cx > 0, hi = cx + 1 < static_cast<uint32_t>(G.mx);
        face(I0{}, BF{}, src(lo, -syz), lo, sx);
        face(I0{}, BT{}, src(hi, syz), hi, sx);
    }
    {
        const bool lo = cy > 0, hi = cy + 1 < static_cast<uint32_t>(G.my);
        face(I1{}, BF{}, src(lo, -G.mz), lo, sy);
        face(I1{}, BT{}, src(hi, G.mz), hi, sy);
    }
    {
        const bool lo = cz > 0, hi = cz + 1 < static_cast<uint32_t>(G.mz);
        face(I2{}, BF{}, src(lo, -1), lo, sz);
        face(I2{}, BT{}, src(hi, 1), hi, sz);
    }
    __builtin_amdgcn_sched_barrier(0);
    lane_apply<N, TC, false, true>([&](int q) { return ldc<TC>(own + (static_cast<int64_t>(q) << lb)); }, R, sx, sy,
                                   sz, acc);
}

// ============================================================ one cell per wave (n >= 5)
// The cell's block lives in an LDS slab (Slab<N> layout, one pencil per lane
// and phase, as in the even-odd wave kernels); the volume product is the
// even-odd LDS apply with the cell-diagonal P_hat, done first.  The six face
// terms are slabs over the two tangential indices, kept in the volume
// product's scratch once that is free: lane (a, b) accumulates alpha and
// beta of every face from the source block's n values along the normal at
// (a, b); the tangential mass M (.) M of all twelve slabs runs as two
// in-place LDS passes of one n-pencil per task (a task owns its row, then
// its column; 12 n tasks per pass spread over the wave); finally lane (j, k)
// adds the face terms to its x-pencil of the volume product.
// The volume product's second scratch slab is the block's own slab s: each
// lane overwrites only the slab positions it has itself just read (its
// pencil in the first phase, its x-pencil in the last), so s, one scratch
// slab and the face slabs are all the LDS a wave needs (10.75 KB at n = 8
// in FP64: 14 waves per CU instead of 11).
template <int N, typename T>
struct WaveLds {
    static constexpr int kT = 12 * N * N > Slab<N>::size ? 12 * N * N : Slab<N>::size;
    T s[Slab<N>::size];          // the cell's block, then its volume product (and scratch t2)
    T t[kT];                     // volume scratch t1, then the twelve face slabs
};

// The lane's x-pencil y[i] = (A u)_c at (i, j, k) with (j, k) = (pc.pa,
// pc.pb), for the active lanes; every lane of the wave must call it.
// TB: ME | MO | PE | PO (even-odd halves of M_hat and of the cell-diagonal
// P_hat); F: endpoint derivatives and the reference penalty.
// HERM: the Hermite-type basis.  The even-odd tables then hold the matrices
// conjugated by D = diag(hermite_sign) (centrosymmetric), so every value is
// multiplied by its sign s(i) s(j) s(k) on load and on store, and the face
// terms read only the layers 0, 1, n-2, n-1 along the normal (the others
// carry no weight: eq. (hermite_traces_3d)).
template <int N, typename T, bool VP, bool HERM = false>
__device__ __forceinline__ void wave_sipg_cell(const T* __restrict__ u, const MeshArgs& G, const T* TB,
                                               const FaceRef<N, T>& F, int64_t c, WaveLds<N, T>& L,
                                               T (&y)[N]) {
    using SL = Slab<N>;
    using S = EOShape<N>;
    constexpr int N3 = N * N * N;
    const T* ME = TB;
    const T* MO = TB + S::SE;
    const T* PE = TB + S::SE + S::SO;
    const T* PO = TB + 2 * S::SE + S::SO;
    const Pencil<N> pc(1);
    const int pa = pc.pa, pb = pc.pb;
    const T* ub = u + G.offset;
    const int lb = G.logB;
    const uint32_t cu = static_cast<uint32_t>(c);
    const uint32_t cz = cu % static_cast<uint32_t>(G.mz);
    const uint32_t rr = cu / static_cast<uint32_t>(G.mz);
    const uint32_t cy = rr % static_cast<uint32_t>(G.my);
    const uint32_t cx = rr / static_cast<uint32_t>(G.my);
    const T sx = static_cast<T>(G.sx), sy = static_cast<T>(G.sy), sz = static_cast<T>(G.sz);
    auto sg = [](int i) { return HERM ? static_cast<T>(hermite_sign(N, i)) : T(1); };
    const T sab = sg(pa) * sg(pb);   // sign of the lane's two tangential indices
    // --- the cell's own block into the slab, volume product in place
    if (pc.act) {
        T x[N];
        pencil_load<N, VP>(x, ub + block_base(c, lb, N3) + (static_cast<int64_t>((pa * N + pb) * N) << lb), lb);
#pragma unroll
        for (int k = 0; k < N; ++k) L.s[SL::at(pa, pb, k)] = HERM ? sab * sg(k) * x[k] : x[k];
    }
    wave_sync();
    eo_apply_lds<N, T>(pc, L.s, L.s, L.t, L.s, ME, MO, PE, PO, sx, sy, sz);   // ends synced
    // --- face slabs in the free scratch: alpha (2 f) and beta (2 f + 1) of
    // face f = 2 axis + upper, slab sl at fs + sl n^2
    T* fs = L.t;
    const int64_t syz = static_cast<int64_t>(G.my) * G.mz;
    auto face = [&](auto Dc, auto UPc, bool interior, int64_t d, T s) {
        constexpr int D = decltype(Dc)::value;
        constexpr bool UP = decltype(UPc)::value;
        constexpr int f = 2 * D + (UP ? 1 : 0);
        const T* w = ub + block_base(interior ? c + d : c, lb, N3);
        const bool first = (UP == interior);
        const T cb0 = first ? T(0.5) * s : T(0);
        const T cbn = first ? T(0) : T(-0.5) * s;
        if (pc.act) {
            // normal to z the n values are the lane's contiguous pencil: one
            // vector load per 16 bytes when VP
            T al = T(0), be = T(0);
            if constexpr (HERM) {
                // two source layers: 0, 1 when the face is interior at the
                // upper end or boundary at the lower end, else n-2, n-1
                // (the weights of the other layers vanish in this basis)
                const int k0 = first ? 0 : N - 2;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int k = k0 + t;
                    T wk = ldc<T>(w + (static_cast<int64_t>(D == 0 ? (k * N + pa) * N + pb
                                                           : D == 1 ? (pa * N + k) * N + pb
                                                                    : (pa * N + pb) * N + k) << lb));
                    wk *= sab * sg(k);
                    // alpha weight of layer k (as below), selected per lane
                    T wgt = T(0);
#pragma unroll
                    for (int kk = 0; kk < N; ++kk) {
                        const T in = UP ? fma(T(-0.5), F.g0[kk], kk == 0 ? -F.sigma : T(0))
                                        : fma(T(0.5), F.g1[kk], kk == N - 1 ? -F.sigma : T(0));
                        const T bd = UP ? T(-0.5) * F.g1[kk] : T(0.5) * F.g0[kk];
                        wgt = kk == k ? s * (interior ? in : bd) : wgt;
                    }
                    al = fma(wgt, wk, al);
                    be = fma(t == 0 ? cb0 : cbn, wk, be);
                }
            } else {
                T wv[N];
                if constexpr (D == 2)
                    pencil_load<N, VP>(wv, w + (static_cast<int64_t>(fq<N, D>(0, pa, pb)) << lb), lb);
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const T in = UP ? fma(T(-0.5), F.g0[k], k == 0 ? -F.sigma : T(0))
                                    : fma(T(0.5), F.g1[k], k == N - 1 ? -F.sigma : T(0));
                    const T bd = UP ? T(-0.5) * F.g1[k] : T(0.5) * F.g0[k];
                    const T wk = D == 2 ? wv[k] : ldc<T>(w + (static_cast<int64_t>(fq<N, D>(k, pa, pb)) << lb));
                    al = fma(s * (interior ? in : bd), wk, al);
                    if (k == 0) be = cb0 * wk;
                    if (k == N - 1) be = fma(cbn, wk, be);
                }
            }
            fs[(2 * f) * N * N + pa * N + pb] = al;
            fs[(2 * f + 1) * N * N + pa * N + pb] = be;
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using BF = std::integral_constant<bool, false>;
    using BT = std::integral_constant<bool, true>;
    face(I0{}, BF{}, cx > 0, -syz, sx);
    face(I0{}, BT{}, cx + 1 < static_cast<uint32_t>(G.mx), syz, sx);
    face(I1{}, BF{}, cy > 0, -static_cast<int64_t>(G.mz), sy);
    face(I1{}, BT{}, cy + 1 < static_cast<uint32_t>(G.my), G.mz, sy);
    face(I2{}, BF{}, cz > 0, -1, sz);
    face(I2{}, BT{}, cz + 1 < static_cast<uint32_t>(G.mz), 1, sz);
    wave_sync();
    // --- tangential mass of the twelve slabs: rows (second index), then columns
    constexpr int HC = S::HC, H = S::H;
    auto mass_pencil = [&](const T (&xin)[N], T (&out)[N]) {
        T e[HC], o[H], E[HC], O[H];
        eo_split<N>(xin, e, o);
        eo_mul<N>(ME, MO, e, o, E, O);
        eo_join<N>(E, O, out);
    };
    for (int task = threadIdx.x; task < 12 * N; task += 64) {
        const int sl = task / N, a = task - (task / N) * N;
        T xin[N], out[N];
#pragma unroll
        for (int b = 0; b < N; ++b) xin[b] = fs[sl * N * N + a * N + b];
        mass_pencil(xin, out);
#pragma unroll
        for (int b = 0; b < N; ++b) fs[sl * N * N + a * N + b] = out[b];
    }
    wave_sync();
    for (int task = threadIdx.x; task < 12 * N; task += 64) {
        const int sl = task / N, b = task - (task / N) * N;
        T xin[N], out[N];
#pragma unroll
        for (int a = 0; a < N; ++a) xin[a] = fs[sl * N * N + a * N + b];
        mass_pencil(xin, out);
#pragma unroll
        for (int a = 0; a < N; ++a) fs[sl * N * N + a * N + b] = out[a];
    }
    wave_sync();
    // --- the lane's x-pencil of the volume product plus the face terms
    if (pc.act) {
        const int j = pa, k = pb;
        T g0j = T(0), g1j = T(0), g0k = T(0), g1k = T(0);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            g0j = j == i ? F.g0[i] : g0j;
            g1j = j == i ? F.g1[i] : g1j;
            g0k = k == i ? F.g0[i] : g0k;
            g1k = k == i ? F.g1[i] : g1k;
        }
        const T ej0 = j == 0 ? T(1) : T(0), ejn = j == N - 1 ? T(1) : T(0);
        const T ek0 = k == 0 ? T(1) : T(0), ekn = k == N - 1 ? T(1) : T(0);
        const T ax0 = fs[0 * N * N + j * N + k], bx0 = fs[1 * N * N + j * N + k];
        const T ax1 = fs[2 * N * N + j * N + k], bx1 = fs[3 * N * N + j * N + k];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T v = L.s[SL::at(i, j, k)];
            v = fma(F.g0[i], bx0, fma(F.g1[i], bx1, v));                       // x faces, beta
            if (i == 0) v += ax0;                                               // x faces, alpha
            if (i == N - 1) v += ax1;
            v = fma(ej0, fs[4 * N * N + i * N + k], v);                             // y faces
            v = fma(g0j, fs[5 * N * N + i * N + k], v);
            v = fma(ejn, fs[6 * N * N + i * N + k], v);
            v = fma(g1j, fs[7 * N * N + i * N + k], v);
            v = fma(ek0, fs[8 * N * N + i * N + j], v);                             // z faces
            v = fma(g0k, fs[9 * N * N + i * N + j], v);
            v = fma(ekn, fs[10 * N * N + i * N + j], v);
            v = fma(g1k, fs[11 * N * N + i * N + j], v);
            y[i] = HERM ? sab * sg(i) * v : v;
        }
    }
    wave_sync();
}

// Tile of workgroup b in an XCD-contiguous order: workgroup b runs on XCD
// b % 8, and each XCD gets a contiguous range of tiles so that the y and z
// neighbours of its tiles share its L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nwg) {
    return (nwg % 8 == 0) ? (b % 8) * (nwg / 8) + b / 8 : b;
}

// Tile of workgroup b for the one-cell-per-lane kernels of a mesh plan (64
// consecutive cells per tile, S tiles per x-plane of cells).  Each XCD again
// gets a contiguous range, but walks it in groups of kLaneSweep consecutive
// tiles carried through the range's rows of S tiles: a tile's x neighbours
// then come kLaneSweep tiles apart in the visiting order instead of S, and
// are still in the XCD's L2 when the second of them reads them.  A
// bijection on [0, nwg): the last group of a row is S mod kLaneSweep wide
// when kLaneSweep does not divide S; the part of the range past its last
// whole row, and meshes whose planes are not whole tiles (S = 0), keep the
// plain order.
constexpr unsigned kLaneSweep = 8;

__device__ __forceinline__ unsigned lane_tile(unsigned b, unsigned nwg, unsigned S) {
    if (nwg % 8 != 0) return b;
    const unsigned L = nwg / 8, base = (b % 8) * L, l = b / 8;
    if (S == 0) return base + l;
    const unsigned R = L / S;
    if (R < 2 || l >= R * S) return base + l;
    const unsigned full = (S / kLaneSweep) * kLaneSweep * R;   // tiles in whole-width groups
    if (l < full) {
        const unsigned chunk = l / (kLaneSweep * R), r = (l / kLaneSweep) % R, g = l % kLaneSweep;
        return base + r * S + chunk * kLaneSweep + g;
    }
    const unsigned w = S % kLaneSweep, e = l - full;          // w > 0 here
    return base + (e / w) * S + (S - w) + e % w;
}

// Row length S for lane_tile: the tiles per x-plane of a mesh plan's cells
// in the Lagrange basis when one plane of blocks (n^3 values of T per cell)
// holds at least twice an XCD's 4 MiB L2, else 0 (plain order).  Measured on
// the coupled operator at n = 4: the grouped order (groups of 8; 4, 16, 32
// and 64 were slower) takes 15% off the time with 8 MiB planes (FP64, 128^2
// cells per plane) and adds 3-6% with 2-4.7 MiB planes; in the Hermite-type
// basis, whose face terms read only two layers of a neighbour, it did not
// pay.  Also 0 when a plane is not whole 64-cell tiles.
template <int N, typename T, bool HERM>
__device__ __forceinline__ unsigned plane_tiles(const MeshArgs& G) {
    constexpr int64_t kMinPlaneBytes = int64_t(8) << 20;
    const int64_t p = static_cast<int64_t>(G.my) * G.mz;
    if (HERM || p % 64 != 0 || p * N * N * N * static_cast<int64_t>(sizeof(T)) < kMinPlaneBytes) return 0u;
    return static_cast<unsigned>(p / 64);
}

// Kernel arguments of a mesh plan's group.
inline MeshArgs mesh_args(const Plan& plan, const GroupInfo& g) {
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
    return G;
}

// 1D tables of the coupled operator: M_hat and the cell-diagonal P_hat
// (A_hat, or A_hat - K_hat for the face part alone), endpoint derivatives and
// the reference penalty.
template <int N, typename TC>
void sipg_tables(const Plan& plan, bool face_only, Pair<N, TC>& R, FaceRef<N, TC>& F) {
    const RefData& ref = plan.ref[N];
    for (int i = 0; i < N * N; ++i) {
        R.m[i] = static_cast<TC>(ref.M[i]);
        R.p[i] = static_cast<TC>(face_only ? ref.A[i] - ref.K[i] : ref.A[i]);
    }
    for (int i = 0; i < N; ++i) {
        F.g0[i] = static_cast<TC>(ref.g0[i]);
        F.g1[i] = static_cast<TC>(ref.g1[i]);
    }
    F.sigma = static_cast<TC>(plan.penalty_C * (N - 1) * N);
}

// The wave kernels of the Hermite-type basis work in the sign-flipped
// coefficients (see wave_sipg_cell): endpoint derivatives D g.
template <int N, typename T>
void flip_face_ref(FaceRef<N, T>& F) {
    for (int k = 0; k < N; ++k) {
        F.g0[k] = static_cast<T>(hermite_sign(N, k)) * F.g0[k];
        F.g1[k] = static_cast<T>(hermite_sign(N, k)) * F.g1[k];
    }
}

}  // namespace tpfdm
