// Lane-per-block device code: one block per lane, all contractions in
// registers (used for n <= 4).
#pragma once

#include "device.h"

namespace tpfdm {

// ============================================================ lane-per-block
// lane_apply streams the block one x-plane (n^2 DoFs) at a time and loads
// plane ip+1 before computing plane ip, so every wave keeps one plane of
// loads in flight while it computes.

// Accumulate acc = A u for one block held by this lane.  load(q) returns DoF
// q of u.  Order: for every x-plane ip of the input, contract z (M and P)
// and y (a = M t, b = s_y P t + s_z M w) inside the plane, then scatter the
// x-contraction into all output planes: 7 n^4 multiply-adds per block.
// ACCUM keeps the incoming acc instead of starting from zero and NEG
// subtracts, so acc = b - A u is formed in place from acc = b.
// FENCE keeps the scheduler from hoisting loads more than one plane ahead
// (for loads from LDS, which it would otherwise issue all at once).
template <int N, typename TC, bool NEG = false, bool ACCUM = false, bool FENCE = false, typename LoadF>
__device__ __forceinline__ void lane_apply(LoadF load, const Pair<N, TC>& R, TC sx, TC sy, TC sz,
                                           TC (&acc)[N * N * N]) {
    constexpr int N2 = N * N;
    if constexpr (!ACCUM) {
#pragma unroll
        for (int q = 0; q < N * N2; ++q) acc[q] = TC(0);
    }
    if constexpr (NEG) sx = -sx;
    TC xb[2][N2];
#pragma unroll
    for (int q = 0; q < N2; ++q) xb[0][q] = load(q);
#pragma unroll
    for (int ip = 0; ip < N; ++ip) {
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
        TC(&x)[N2] = xb[ip & 1];
        if (ip + 1 < N) {
#pragma unroll
            for (int q = 0; q < N2; ++q) xb[(ip + 1) & 1][q] = load((ip + 1) * N2 + q);
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            TC t[N], w[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                TC st = TC(0), sw = TC(0);
#pragma unroll
                for (int kk = 0; kk < N; ++kk) {
                    st = fma(R.m[k * N + kk], x[j * N + kk], st);
                    sw = fma(R.p[k * N + kk], x[j * N + kk], sw);
                }
                t[j] = st;
                w[j] = sw;
            }
#pragma unroll
            for (int j = 0; j < N; ++j) {
                TC a = TC(0), b1 = TC(0), b2 = TC(0);
#pragma unroll
                for (int jj = 0; jj < N; ++jj) {
                    a = fma(R.m[j * N + jj], t[jj], a);
                    b1 = fma(R.p[j * N + jj], t[jj], b1);
                    b2 = fma(R.m[j * N + jj], w[jj], b2);
                }
                a *= sx;
                TC b = fma(sy, b1, sz * b2);
                if constexpr (NEG) b = -b;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    TC& o = acc[(i * N + j) * N + k];
                    o = fma(R.p[i * N + ip], a, fma(R.m[i * N + ip], b, o));
                }
            }
        }
    }
}

// x <- D^{-1} x for one block held entirely in this lane's registers, in
// place with N temporaries per pencil: S^T along z, y and x, the diagonal
// scaling by 1/(lam_i s_x + lam_j s_y + lam_k s_z), then S along x, y and z
// (6 n^4 multiply-adds and n^3 reciprocals).  Only one block-sized array is
// live, so a lane holds the n = 4 FP64 block in 128 VGPRs plus temporaries.
template <int N, typename TC>
__device__ __forceinline__ void lane_fdm_inplace(TC (&v)[N * N * N], const Eig<N, TC>& E, TC sx, TC sy, TC sz) {
    constexpr int N2 = N * N;
    // forward transform of the pencil (base, base + st, ...): v_c <- sum_k S[k][c] v_k
    auto fwd = [&](int base, int st) {
        TC t[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            TC a = TC(0);
#pragma unroll
            for (int k = 0; k < N; ++k) a = fma(E.s[k * N + c], v[base + k * st], a);
            t[c] = a;
        }
#pragma unroll
        for (int c = 0; c < N; ++c) v[base + c * st] = t[c];
    };
    // backward transform: v_k <- sum_c S[k][c] v_c
    auto bwd = [&](int base, int st) {
        TC t[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            TC a = TC(0);
#pragma unroll
            for (int c = 0; c < N; ++c) a = fma(E.s[k * N + c], v[base + c * st], a);
            t[k] = a;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) v[base + k * st] = t[k];
    };
#pragma unroll
    for (int p = 0; p < N2; ++p) fwd(p * N, 1);                      // z: (i, j) pencils
#pragma unroll
    for (int p = 0; p < N2; ++p) fwd((p / N) * N2 + (p % N), N);     // y: (i, k) pencils
#pragma unroll
    for (int p = 0; p < N2; ++p) fwd(p, N2);                         // x: (j, k) pencils
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const TC mu = fma(E.lam[i], sx, E.lam[j] * sy);
#pragma unroll
            for (int k = 0; k < N; ++k) v[(i * N + j) * N + k] *= recip(fma(E.lam[k], sz, mu));
        }
#pragma unroll
    for (int p = 0; p < N2; ++p) bwd(p, N2);
#pragma unroll
    for (int p = 0; p < N2; ++p) bwd((p / N) * N2 + (p % N), N);
#pragma unroll
    for (int p = 0; p < N2; ++p) bwd(p * N, 1);
}

// Symmetry classes of a symmetric, centrosymmetric N x N matrix
// (A[i][j] = A[j][i] = A[N-1-i][N-1-j]): rep[e] is the row-major index of
// the first entry of e's class.  Reading a table through rep lets the
// compiler keep one scalar register per distinct value.
template <int N>
struct SymOrbits {
    int rep[N * N];
    constexpr SymOrbits() : rep() {
        for (int e = 0; e < N * N; ++e) rep[e] = -1;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                if (rep[i * N + j] >= 0) continue;
                const int c = i * N + j;
                rep[i * N + j] = c;
                rep[j * N + i] = c;
                rep[(N - 1 - i) * N + (N - 1 - j)] = c;
                rep[(N - 1 - j) * N + (N - 1 - i)] = c;
            }
    }
};

// (M_hat, P_hat) read through their symmetry classes from full row-major
// tables (kernel arguments or memory).
template <int N, typename T, typename Src>
__device__ __forceinline__ Pair<N, T> sym_pair(const Src* m, const Src* p) {
    constexpr SymOrbits<N> O;
    Pair<N, T> R;
#pragma unroll
    for (int e = 0; e < N * N; ++e) {
        R.m[e] = static_cast<T>(m[O.rep[e]]);
        R.p[e] = static_cast<T>(p[O.rep[e]]);
    }
    return R;
}
template <int N>
__device__ __forceinline__ Pair<N, double> sym_pair(const double (&m)[N * N], const double (&p)[N * N]) {
    return sym_pair<N, double, double>(&m[0], &p[0]);
}

// One tile (64 consecutive blocks, one per lane) of the block-local
// iterative refinement:
//   r = b - D x (FP64), s = ||r||_inf, d = D~^{-1}(r / s) in precision TI
//   (rounded to FP16/BF16 on input and output for RND), x <- x + s d (FP64),
// until ||r||_2 <= rtol ||b||_2 or maxit corrections.  x lives in LDS (xs,
// lane-interleaved, conflict-free), r and d in registers; b is re-read from
// global memory for every residual (cached loads: it stays in L2/MALL), so
// the register file holds one block-sized array at a time.  A residual of an
// all-zero x is b itself: the first product is skipped when every x of the
// wave is zero on entry.  NT: the vectors' rows are whole cache lines; LB:
// log2 of the layout width when known at compile time (-1: G.logB), which
// turns the n^3 element offsets into constants instead of scalar registers.
template <int N, typename TI, int RND, bool NT, int LB = -1>
__device__ __forceinline__ void lane_solve_tile(const double* __restrict__ b, double* __restrict__ x, const GArgs& G,
                                                const Pair<N, double>& RA, const Eig<N, TI>& E, int64_t t,
                                                double rtol, int maxit, int32_t* __restrict__ iters,
                                                double* __restrict__ relres, int64_t block0, SolveAcc& acc,
                                                double (*xs)[64]) {
    constexpr int N3 = N * N * N;
    const int lane = threadIdx.x;
    const int64_t g = t * 64 + lane;
    const bool valid = g < G.nblocks;
    const int lb = LB >= 0 ? LB : G.logB;
    // lanes past the end read block 0 (in bounds) and discard it: the
    // loads stay unconditional, with no branch per element
    const int64_t base = G.offset + block_base(valid ? g : 0, lb, N3);
    const double* bb = b + base;
    double* xb = x + base;
    double sx = 1.0, sy = 1.0, sz = 1.0;
    if (valid) block_scales(G.h, g, sx, sy, sz);
    bool nz = false;
#pragma unroll 8
    for (int q = 0; q < N3; ++q) {
        const double xl = ldv<NT, double>(xb + (static_cast<int64_t>(q) << lb));
        const double xv = valid ? xl : 0.0;
        xs[q][lane] = xv;
        nz = nz || xv != 0.0;
    }
    double r[N3];
    double bn = 0.0;
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        const double bl = ldc<double>(bb + (static_cast<int64_t>(q) << lb));
        const double bv = valid ? bl : 0.0;
        r[q] = bv;
        bn = fma(bv, bv, bn);
    }
    if (bn == 0.0) {  // b = 0: x = 0 after no correction
#pragma unroll
        for (int q = 0; q < N3; ++q) xs[q][lane] = 0.0;
        nz = false;
    }
    int it = 0;
    double rel = 0.0;
    bool done = !valid;
    for (bool first = true;; first = false) {
        if (!first) {
#pragma unroll
            for (int q = 0; q < N3; ++q) {
                const double bl = ldc<double>(bb + (static_cast<int64_t>(q) << lb));
                r[q] = valid ? bl : 0.0;
            }
        }
        if (!first || __any(nz))
            lane_apply<N, double, true, true, true>([&](int q) { return xs[q][lane]; }, RA, sx, sy, sz, r);
        double rr = 0.0, rmax = 0.0;
#pragma unroll
        for (int q = 0; q < N3; ++q) {
            rr = fma(r[q], r[q], rr);
            rmax = fmax(rmax, fabs(r[q]));
        }
        if (!done) {
            rel = bn == 0.0 ? 0.0 : sqrt(rr / bn);
            done = !(rel > rtol) || it >= maxit;
        }
        if (__all(done)) break;
        const double s = done ? 0.0 : rmax;
        const double inv_s = s > 0.0 ? 1.0 / s : 0.0;
        TI d[N3];  // scaled residual in the inner precision; r is dead from here on
#pragma unroll
        for (int q = 0; q < N3; ++q) d[q] = round_to<RND>(static_cast<TI>(r[q] * inv_s));
        // the n^3 eigenvalue scalings are loop-invariant; recomputing them per
        // correction is cheaper than the registers the compiler would hold
        // them in across the loop (an empty asm makes the scalings opaque)
        TI fsx = static_cast<TI>(sx), fsy = static_cast<TI>(sy), fsz = static_cast<TI>(sz);
        asm volatile("" : "+v"(fsx), "+v"(fsy), "+v"(fsz));
        lane_fdm_inplace<N, TI>(d, E, fsx, fsy, fsz);
#pragma unroll
        for (int q = 0; q < N3; ++q) xs[q][lane] = fma(s, static_cast<double>(round_to<RND>(d[q])), xs[q][lane]);
        if (!done) ++it;
    }
    if (valid) {
#pragma unroll 8
        for (int q = 0; q < N3; ++q) stv<NT>(xb + (static_cast<int64_t>(q) << lb), xs[q][lane]);
        if (iters) iters[block0 + g] = it;
        if (relres) relres[block0 + g] = rel;
        acc.add(it, rel, rtol);
    }
}

}  // namespace tpfdm
