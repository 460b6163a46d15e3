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
#include "device.h"

namespace tpfdm {

// ============================================================ lane-per-block
// Both transforms below stream the block one x-plane (n^2 DoFs) at a time and
// load plane ip+1 before computing plane ip, so every wave keeps one plane of
// loads in flight while it computes.

// Accumulate acc = A u for one block held by this lane.  load(q) returns DoF
// q of u.  Order: for every x-plane ip of the input, contract z (M and P)
// and y (a = M t, b = s_y P t + s_z M w) inside the plane, then scatter the
// x-contraction into all output planes: 7 n^4 multiply-adds per block.
template <int N, typename TC, typename LoadF>
__device__ __forceinline__ void lane_apply(LoadF load, const Pair<N, TC>& R, TC sx, TC sy, TC sz,
                                           TC (&acc)[N * N * N]) {
    constexpr int N2 = N * N;
#pragma unroll
    for (int q = 0; q < N * N2; ++q) acc[q] = TC(0);
    TC xb[2][N2];
#pragma unroll
    for (int q = 0; q < N2; ++q) xb[0][q] = load(q);
#pragma unroll
    for (int ip = 0; ip < N; ++ip) {
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
                const TC b = fma(sy, b1, sz * b2);
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    TC& o = acc[(i * N + j) * N + k];
                    o = fma(R.p[i * N + ip], a, fma(R.m[i * N + ip], b, o));
                }
            }
        }
    }
}

// D^{-1} r for one block held by this lane; load(q) reads r, emit(q, v)
// consumes output DoF q.  Forward transform S^T plane by plane accumulated
// into y, diagonal scaling by 1/(lam_i s_x + lam_j s_y + lam_k s_z), then
// (S (x) S) in place on every plane of y and finally the x-contraction, one
// output DoF at a time: 6 n^4 multiply-adds and n^3 reciprocals per block.
template <int N, typename TC, typename LoadF, typename EmitF>
__device__ __forceinline__ void lane_inverse(LoadF load, EmitF emit, const Eig<N, TC>& E, TC sx, TC sy,
                                             TC sz) {
    constexpr int N2 = N * N;
    TC y[N * N2];
#pragma unroll
    for (int q = 0; q < N * N2; ++q) y[q] = TC(0);
    TC xb[2][N2];
#pragma unroll
    for (int q = 0; q < N2; ++q) xb[0][q] = load(q);
#pragma unroll
    for (int ip = 0; ip < N; ++ip) {
        TC(&x)[N2] = xb[ip & 1];
        if (ip + 1 < N) {
#pragma unroll
            for (int q = 0; q < N2; ++q) xb[(ip + 1) & 1][q] = load((ip + 1) * N2 + q);
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            TC t[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                TC s = TC(0);
#pragma unroll
                for (int kk = 0; kk < N; ++kk) s = fma(E.s[kk * N + k], x[j * N + kk], s);
                t[j] = s;
            }
#pragma unroll
            for (int j = 0; j < N; ++j) {
                TC a = TC(0);
#pragma unroll
                for (int jj = 0; jj < N; ++jj) a = fma(E.s[jj * N + j], t[jj], a);
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    TC& o = y[(i * N + j) * N + k];
                    o = fma(E.s[ip * N + i], a, o);
                }
            }
        }
    }
    TC lx[N], ly[N], lz[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        lx[i] = E.lam[i] * sx;
        ly[i] = E.lam[i] * sy;
        lz[i] = E.lam[i] * sz;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int k = 0; k < N; ++k) y[(i * N + j) * N + k] *= recip(lx[i] + ly[j] + lz[k]);
    // (S (x) S) on every x-plane of y, in place
#pragma unroll
    for (int a = 0; a < N; ++a) {
        TC z[N2];
#pragma unroll
        for (int bq = 0; bq < N; ++bq)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                TC s = TC(0);
#pragma unroll
                for (int c = 0; c < N; ++c) s = fma(E.s[k * N + c], y[a * N2 + bq * N + c], s);
                z[bq * N + k] = s;
            }
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                TC s = TC(0);
#pragma unroll
                for (int bq = 0; bq < N; ++bq) s = fma(E.s[j * N + bq], z[bq * N + k], s);
                y[a * N2 + j * N + k] = s;
            }
    }
    // x-contraction, one output DoF at a time
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int q = 0; q < N2; ++q) {
            TC s = TC(0);
#pragma unroll
            for (int a = 0; a < N; ++a) s = fma(E.s[i * N + a], y[a * N2 + q], s);
            emit(i * N2 + q, s);
        }
}

template <int N, typename TS, typename TC>
__global__ __launch_bounds__(256, 2) void k_apply_lane(const TS* __restrict__ u, TS* __restrict__ v, GArgs G,
                                                    Pair<N, TC> R) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G.nblocks) return;
    const int64_t base = G.offset + block_base(g, G.logB, N * N * N);
    const TS* ub = u + base;
    TS* vb = v + base;
    const int lb = G.logB;
    TC sx, sy, sz;
    block_scales(G.h, g, sx, sy, sz);
    TC acc[N * N * N];
    lane_apply<N, TC>([&](int q) { return ldc<TC>(ub + (static_cast<int64_t>(q) << lb)); }, R, sx, sy, sz,
                      acc);
#pragma unroll
    for (int q = 0; q < N * N * N; ++q) stc(vb + (static_cast<int64_t>(q) << lb), acc[q]);
}

template <int N, typename TS, typename TC>
__global__ __launch_bounds__(256, 2) void k_inverse_lane(const TS* __restrict__ r, TS* __restrict__ x, GArgs G,
                                                      Eig<N, TC> E) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= G.nblocks) return;
    const int64_t base = G.offset + block_base(g, G.logB, N * N * N);
    const TS* rb = r + base;
    TS* xb = x + base;
    const int lb = G.logB;
    TC sx, sy, sz;
    block_scales(G.h, g, sx, sy, sz);
    lane_inverse<N, TC>([&](int q) { return ldc<TC>(rb + (static_cast<int64_t>(q) << lb)); },
                        [&](int q, TC val) { stc(xb + (static_cast<int64_t>(q) << lb), val); }, E, sx, sy, sz);
}

__device__ __forceinline__ void record_solve(SolveSummary* sum, int32_t* iters, double* relres, int64_t gidx,
                                             int it, double rel, double rtol) {
    if (iters) iters[gidx] = it;
    if (relres) relres[gidx] = rel;
    if (sum) {
        const bool finite = (rel == rel) && rel <= 1.7976931348623157e308;
        atomicMax(&sum->max_iters, it);
        if (!(rel <= rtol)) atomicAdd(&sum->n_failed, 1);
        if (!finite) atomicAdd(&sum->nonfinite, 1);
        atomicMax(&sum->max_relres_bits, static_cast<unsigned long long>(__double_as_longlong(rel)));
    }
}

// ============================================================ wave-per-tile
// dst = A src on the lane's LDS slab (dst may alias src); t1, t2 scratch
// slabs.  Lane (i,j) contracts z, lane (i,k) contracts y, lane (j,k)
// contracts x; within a phase each lane reads and writes only its pencil.
template <int N, typename TC>
__device__ __forceinline__ void wave_apply(const Pencil<N>& pc, const TC* src, TC* dst, TC* t1, TC* t2,
                                           const Pair<N, TC>& R, TC sx, TC sy, TC sz) {
    using L = Slab<N>;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {
        TC x[N];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = src[L::at(pa, pb, k)];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            TC st = TC(0), sw = TC(0);
#pragma unroll
            for (int kk = 0; kk < N; ++kk) {
                st = fma(R.m[k * N + kk], x[kk], st);
                sw = fma(R.p[k * N + kk], x[kk], sw);
            }
            t1[L::at(pa, pb, k)] = st;
            t2[L::at(pa, pb, k)] = sw;
        }
    }
    __syncthreads();
    if (pc.act) {
        TC t[N], w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            t[j] = t1[L::at(pa, j, pb)];
            w[j] = t2[L::at(pa, j, pb)];
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
            t1[L::at(pa, j, pb)] = a * sx;
            t2[L::at(pa, j, pb)] = fma(sy, b1, sz * b2);
        }
    }
    __syncthreads();
    if (pc.act) {
        TC a[N], b[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            a[i] = t1[L::at(i, pa, pb)];
            b[i] = t2[L::at(i, pa, pb)];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            TC o = TC(0);
#pragma unroll
            for (int ii = 0; ii < N; ++ii) o = fma(R.p[i * N + ii], a[ii], fma(R.m[i * N + ii], b[ii], o));
            dst[L::at(i, pa, pb)] = o;
        }
    }
    __syncthreads();
}

// slab <- D^{-1} slab in place on the lane's LDS slab (t1 scratch slab).
template <int N, typename TC>
__device__ __forceinline__ void wave_inverse(const Pencil<N>& pc, TC* slab, TC* t1, const Eig<N, TC>& E, TC sx,
                                             TC sy, TC sz) {
    using L = Slab<N>;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {  // z forward: lane (i, j)
        TC x[N];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = slab[L::at(pa, pb, k)];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            TC s = TC(0);
#pragma unroll
            for (int k = 0; k < N; ++k) s = fma(E.s[k * N + c], x[k], s);
            t1[L::at(pa, pb, c)] = s;
        }
    }
    __syncthreads();
    if (pc.act) {  // y forward: lane (i, c)
        TC t[N];
#pragma unroll
        for (int j = 0; j < N; ++j) t[j] = t1[L::at(pa, j, pb)];
#pragma unroll
        for (int bq = 0; bq < N; ++bq) {
            TC s = TC(0);
#pragma unroll
            for (int j = 0; j < N; ++j) s = fma(E.s[j * N + bq], t[j], s);
            t1[L::at(pa, bq, pb)] = s;
        }
    }
    __syncthreads();
    if (pc.act) {  // x forward, diagonal scaling, x backward: lane (b, c)
        TC t[N], y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) t[i] = t1[L::at(i, pa, pb)];
        const TC mu_bc = E.lam[pa] * sy + E.lam[pb] * sz;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            TC s = TC(0);
#pragma unroll
            for (int i = 0; i < N; ++i) s = fma(E.s[i * N + a], t[i], s);
            y[a] = s * recip(fma(E.lam[a], sx, mu_bc));
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            TC s = TC(0);
#pragma unroll
            for (int a = 0; a < N; ++a) s = fma(E.s[i * N + a], y[a], s);
            t1[L::at(i, pa, pb)] = s;
        }
    }
    __syncthreads();
    if (pc.act) {  // y backward: lane (i, c)
        TC t[N];
#pragma unroll
        for (int bq = 0; bq < N; ++bq) t[bq] = t1[L::at(pa, bq, pb)];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            TC s = TC(0);
#pragma unroll
            for (int bq = 0; bq < N; ++bq) s = fma(E.s[j * N + bq], t[bq], s);
            t1[L::at(pa, j, pb)] = s;
        }
    }
    __syncthreads();
    if (pc.act) {  // z backward: lane (i, j)
        TC t[N];
#pragma unroll
        for (int c = 0; c < N; ++c) t[c] = t1[L::at(pa, pb, c)];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            TC s = TC(0);
#pragma unroll
            for (int c = 0; c < N; ++c) s = fma(E.s[k * N + c], t[c], s);
            slab[L::at(pa, pb, k)] = s;
        }
    }
    __syncthreads();
}

// Global <-> LDS staging of the tile's blocks: consecutive lanes take
// consecutive DoFs of a block, so each wave access is one coalesced segment
// when B = 1 (block-contiguous layout).
template <int N, typename TS, typename TC>
__device__ __forceinline__ void stage_in(const TS* __restrict__ src, TC* slabs, const GArgs& G, int64_t g0,
                                         int nvalid) {
    using L = Slab<N>;
    for (int e = threadIdx.x; e < nvalid * L::N3; e += 64) {
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        slabs[w * L::size + L::lin(q)] =
            ldc<TC>(src + G.offset + block_base(g0 + w, G.logB, L::N3) + (static_cast<int64_t>(q) << G.logB));
    }
}
template <int N, typename TS, typename TC>
__device__ __forceinline__ void stage_out(TS* __restrict__ dst, const TC* slabs, const GArgs& G, int64_t g0,
                                          int nvalid) {
    using L = Slab<N>;
    for (int e = threadIdx.x; e < nvalid * L::N3; e += 64) {
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        stc(dst + G.offset + block_base(g0 + w, G.logB, L::N3) + (static_cast<int64_t>(q) << G.logB),
            slabs[w * L::size + L::lin(q)]);
    }
}

// Block-local iterative refinement (a6), one wave per tile of BPW blocks:
//   r = b - D x (FP64), s = ||r||_inf, d = D~^{-1} (r / s) in precision TI,
//   x <- x + s d (FP64), until ||r||_2 <= rtol ||b||_2 or maxit corrections.
// x and b stay in LDS for all iterations (b read once, x written once).
// Per-block norms are reduced over the block's pencils through LDS.
template <int N, typename TI>
__global__ __launch_bounds__(64) void k_solve_wave(const double* __restrict__ b, double* __restrict__ x, GArgs G,
                                                   Pair<N, double> R, Eig<N, TI> E, double rtol, int maxit,
                                                   int32_t* __restrict__ iters, double* __restrict__ relres,
                                                   int64_t block0, SolveSummary* sum) {
    using L = Slab<N>;
    constexpr int SZ = L::BPW * L::size;
    __shared__ double xs[SZ], bs[SZ], ra[SZ], t1[SZ], t2[SZ];
    __shared__ TI rs[SZ], ti[SZ];
    __shared__ double part[2][64];
    __shared__ double red[3][L::BPW];
    __shared__ int done[L::BPW];
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * L::BPW;
    if (g0 >= G.nblocks) return;
    const int nvalid = static_cast<int>(G.nblocks - g0 < L::BPW ? G.nblocks - g0 : L::BPW);
    stage_in<N>(b, bs, G, g0, nvalid);
    stage_in<N>(x, xs, G, g0, nvalid);
    const Pencil<N> pc(nvalid);
    const int lane = threadIdx.x;
    const int wl = pc.w < L::BPW ? pc.w : 0;
    const int so = wl * L::size;
    double sx = 1.0, sy = 1.0, sz = 1.0;
    if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
    const TI sxi = static_cast<TI>(sx), syi = static_cast<TI>(sy), szi = static_cast<TI>(sz);
    __syncthreads();
    // ||b||^2 per block: each lane sums its z-pencil, then pencil 0 of the
    // block sums the block's lanes.
    double acc = 0.0;
    if (pc.act)
        for (int k = 0; k < N; ++k) {
            const double bv = bs[so + L::at(pc.pa, pc.pb, k)];
            acc = fma(bv, bv, acc);
        }
    part[0][lane] = acc;
    __syncthreads();
    if (pc.act && pc.pa == 0 && pc.pb == 0) {
        double s = 0.0;
        for (int l = 0; l < L::N2; ++l) s += part[0][lane + l];
        red[0][pc.w] = s;
        red[1][pc.w] = 0.0;
        done[pc.w] = 0;
    }
    __syncthreads();
    int it = 0;  // identical on all lanes of a block
    const double bn = pc.act ? red[0][pc.w] : 0.0;
    double rel = 0.0;
    if (pc.act && bn == 0.0)
        for (int k = 0; k < N; ++k) xs[so + L::at(pc.pa, pc.pb, k)] = 0.0;
    for (;;) {
        wave_apply<N, double>(pc, xs + so, ra + so, t1 + so, t2 + so, R, sx, sy, sz);
        double rr = 0.0, rmax = 0.0;
        if (pc.act)
            for (int k = 0; k < N; ++k) {
                const int a = so + L::at(pc.pa, pc.pb, k);
                const double rv = bs[a] - ra[a];
                ra[a] = rv;
                rr = fma(rv, rv, rr);
                rmax = fmax(rmax, fabs(rv));
            }
        part[0][lane] = rr;
        part[1][lane] = rmax;
        __syncthreads();
        if (pc.act && pc.pa == 0 && pc.pb == 0) {
            double s = 0.0, m = 0.0;
            for (int l = 0; l < L::N2; ++l) {
                s += part[0][lane + l];
                m = fmax(m, part[1][lane + l]);
            }
            red[1][pc.w] = s;
            red[2][pc.w] = m;
        }
        __syncthreads();
        bool mine_done = true;
        if (pc.act && !done[pc.w]) {
            rel = bn == 0.0 ? 0.0 : sqrt(red[1][pc.w] / bn);
            mine_done = !(rel > rtol) || it >= maxit;
        }
        __syncthreads();
        if (pc.act && pc.pa == 0 && pc.pb == 0 && mine_done) done[pc.w] = 1;
        // the wave continues while any block still iterates
        const bool any_left = __any(pc.act && !mine_done);
        if (!any_left) break;
        // scaled residual r / s in the inner precision (finished blocks get 0)
        const double rmax_b = pc.act ? red[2][pc.w] : 0.0;
        const double inv_s = (pc.act && !mine_done && rmax_b > 0.0) ? 1.0 / rmax_b : 0.0;
        if (pc.act)
            for (int k = 0; k < N; ++k) {
                const int a = so + L::at(pc.pa, pc.pb, k);
                rs[a] = static_cast<TI>(ra[a] * inv_s);
            }
        __syncthreads();
        wave_inverse<N, TI>(pc, rs + so, ti + so, E, sxi, syi, szi);
        if (pc.act && !mine_done) {
            for (int k = 0; k < N; ++k) {
                const int a = so + L::at(pc.pa, pc.pb, k);
                xs[a] = fma(rmax_b, static_cast<double>(rs[a]), xs[a]);
            }
            ++it;
        }
        __syncthreads();
    }
    __syncthreads();
    stage_out<N>(x, xs, G, g0, nvalid);
    if (pc.act && pc.pa == 0 && pc.pb == 0) record_solve(sum, iters, relres, block0 + g0 + pc.w, it, rel, rtol);
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

__global__ void k_summary_reset(SolveSummary* s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        s->max_iters = 0;
        s->n_failed = 0;
        s->nonfinite = 0;
        s->pad = 0;
        s->max_relres_bits = 0ull;
    }
}

// ============================================================ host launchers
namespace {

constexpr int kLaneThreads = 256;

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

template <int N>
unsigned wave_tiles(const GroupInfo& g) {
    return static_cast<unsigned>((g.nblocks + Slab<N>::BPW - 1) / Slab<N>::BPW);
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
    hipLaunchKernelGGL((k_apply_lane<N, TS, TC>), dim3(grid), dim3(kLaneThreads), 0, s,
                       static_cast<const TS*>(u), static_cast<TS*>(v), gargs(g), R);
    return check_launch("apply launch");
}

template <int N, typename TS, typename TC>
tp_status inverse_n(const GroupInfo& g, const RefData& ref, const void* r, void* x, hipStream_t s) {
    const auto E = make_eig<N, TC>(ref);
    const unsigned grid = static_cast<unsigned>((g.nblocks + kLaneThreads - 1) / kLaneThreads);
    hipLaunchKernelGGL((k_inverse_lane<N, TS, TC>), dim3(grid), dim3(kLaneThreads), 0, s,
                       static_cast<const TS*>(r), static_cast<TS*>(x), gargs(g), E);
    return check_launch("apply_inverse launch");
}

template <int N, typename TI>
tp_status solve_n(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                  int32_t* iters, double* relres, hipStream_t s) {
    const RefData& ref = plan.ref[N];
    const auto R = make_pair<N, double>(ref.M, ref.A);
    const auto E = make_eig<N, TI>(ref);
    SolveSummary* sum = static_cast<SolveSummary*>(plan.summary_dev);
    hipLaunchKernelGGL((k_solve_wave<N, TI>), dim3(wave_tiles<N>(g)), dim3(64), 0, s, b, x, gargs(g), R, E, rtol,
                       maxit, iters, relres, g.block0, sum);
    return check_launch("solve launch");
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

template <typename TI>
tp_status solve_dispatch(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                         int32_t* iters, double* relres, hipStream_t s) {
    switch (g.n) {
        case 2: return solve_n<2, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case 3: return solve_n<3, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case 4: return solve_n<4, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case 5: return solve_n<5, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case 6: return solve_n<6, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case 7: return solve_n<7, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case 8: return solve_n<8, TI>(plan, g, b, x, rtol, maxit, iters, relres, s);
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

tp_status launch_solve(const Plan& plan, const GroupInfo& g, const double* b, double* x, tp_dtype inner,
                       double rtol, int maxit, int32_t* iters, double* relres, hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    switch (inner) {
        case TP_F64: return solve_dispatch<double>(plan, g, b, x, rtol, maxit, iters, relres, s);
        case TP_F32: return solve_dispatch<float>(plan, g, b, x, rtol, maxit, iters, relres, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "solve inner precision must be TP_F64 or TP_F32");
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

tp_status launch_summary_reset(void* summary_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_summary_reset, dim3(1), dim3(64), 0, s, static_cast<SolveSummary*>(summary_dev));
    return check_launch("summary reset");
}

}  // namespace tpfdm
