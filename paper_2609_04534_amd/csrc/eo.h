// Even-odd device code for the wave-per-tile kernels (see eo.hip).
#pragma once

#include <type_traits>

#include "device.h"

namespace tpfdm {

template <int N>
struct EOShape {
    static constexpr int H = N / 2;
    static constexpr int HC = (N + 1) / 2;
    static constexpr int SE = HC * HC;
    static constexpr int SO = H * H;
};

// e, o parts of a pencil.
template <int N, typename T>
__device__ __forceinline__ void eo_split(const T (&x)[N], T (&e)[EOShape<N>::HC], T (&o)[EOShape<N>::H]) {
    constexpr int H = EOShape<N>::H;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        e[j] = x[j] + x[N - 1 - j];
        o[j] = x[j] - x[N - 1 - j];
    }
    if constexpr (N % 2 == 1) e[H] = x[H];
}

// E = AE e (HC outputs), O = AO o (H outputs); matrices row-major.
template <int N, typename T>
__device__ __forceinline__ void eo_mul(const T* AE, const T* AO, const T (&e)[EOShape<N>::HC],
                                       const T (&o)[EOShape<N>::H], T (&E)[EOShape<N>::HC],
                                       T (&O)[EOShape<N>::H]) {
    constexpr int H = EOShape<N>::H, HC = EOShape<N>::HC;
#pragma unroll
    for (int i = 0; i < HC; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < HC; ++j) s = fma(AE[i * HC + j], e[j], s);
        E[i] = s;
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < H; ++j) s = fma(AO[i * H + j], o[j], s);
        O[i] = s;
    }
}

template <int N, typename T>
__device__ __forceinline__ void eo_join(const T (&E)[EOShape<N>::HC], const T (&O)[EOShape<N>::H], T (&y)[N]) {
    constexpr int H = EOShape<N>::H;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        y[i] = E[i] + O[i];
        y[N - 1 - i] = E[i] - O[i];
    }
    if constexpr (N % 2 == 1) y[H] = E[H];
}

// Forward spectral transform y = S^T x along a pencil: the first HC outputs
// are the coefficients of the symmetric eigenvectors, the last H those of
// the antisymmetric ones (SE[k][c] = S[k][sym c] for k < HC, SO likewise).
template <int N, typename T>
__device__ __forceinline__ void eo_fwd(const T* SE, const T* SO, const T (&x)[N], T (&y)[N]) {
    constexpr int H = EOShape<N>::H, HC = EOShape<N>::HC;
    T e[HC], o[H];
    eo_split<N>(x, e, o);
#pragma unroll
    for (int c = 0; c < HC; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < HC; ++k) s = fma(SE[k * HC + c], e[k], s);
        y[c] = s;
    }
#pragma unroll
    for (int c = 0; c < H; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < H; ++k) s = fma(SO[k * H + c], o[k], s);
        y[HC + c] = s;
    }
}

// Backward transform x = S y (y in the split spectral order of eo_fwd).
template <int N, typename T>
__device__ __forceinline__ void eo_bwd(const T* SE, const T* SO, const T (&y)[N], T (&x)[N]) {
    constexpr int H = EOShape<N>::H, HC = EOShape<N>::HC;
    T E[HC], O[H];
#pragma unroll
    for (int k = 0; k < HC; ++k) {
        T s = T(0);
#pragma unroll
        for (int c = 0; c < HC; ++c) s = fma(SE[k * HC + c], y[c], s);
        E[k] = s;
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
        T s = T(0);
#pragma unroll
        for (int c = 0; c < H; ++c) s = fma(SO[k * H + c], y[HC + c], s);
        O[k] = s;
    }
    eo_join<N>(E, O, x);
}

// ------------------------------------------------------------ pencil I/O
// Lane (w, i, j) of a tile owns the z-pencil (i, j, 0..n-1) of block w.  For
// the block-contiguous layout (B = 1) a pencil is n consecutive elements and
// is moved with 16-byte vector accesses when the address allows it.
template <int N, typename TS>
__device__ __forceinline__ const TS* pencil_ptr(const TS* base, const GArgs& G, int64_t g, int i, int j) {
    return base + G.offset + block_base(g, G.logB, N * N * N) + (static_cast<int64_t>((i * N + j) * N) << G.logB);
}

// 16 bytes of storage elements.
template <typename TS>
union Pack16 {
    static constexpr int n = 16 / static_cast<int>(sizeof(TS));
    uint4 u;
    TS s[16 / sizeof(TS)];
};

// With VP the caller guarantees B = 1 and 16-byte aligned pencils.
template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void pencil_load(TC (&x)[N], const TS* __restrict__ p, int logB) {
    constexpr int VEC = Pack16<TS>::n;
    if constexpr (VP && N % VEC == 0) {
        {
            const uint4* vp = reinterpret_cast<const uint4*>(p);
#pragma unroll
            for (int c = 0; c < N / VEC; ++c) {
                Pack16<TS> pk;
                pk.u = vp[c];
#pragma unroll
                for (int l = 0; l < VEC; ++l) x[c * VEC + l] = ldc<TC>(&pk.s[l]);
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = ldc<TC>(p + (static_cast<int64_t>(k) << logB));
}

template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void pencil_store(TS* __restrict__ p, const TC (&x)[N], int logB) {
    constexpr int VEC = Pack16<TS>::n;
    if constexpr (VP && N % VEC == 0) {
        {
            uint4* vp = reinterpret_cast<uint4*>(p);
#pragma unroll
            for (int c = 0; c < N / VEC; ++c) {
                Pack16<TS> pk;
#pragma unroll
                for (int l = 0; l < VEC; ++l) stc(&pk.s[l], x[c * VEC + l]);
                vp[c] = pk.u;
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) stc(p + (static_cast<int64_t>(k) << logB), x[k]);
}

template <int N>
__device__ __forceinline__ int nvalid_of(const GArgs& G, int64_t t) {
    const int64_t g0 = t * Slab<N>::BPW;
    return static_cast<int>(G.nblocks - g0 < Slab<N>::BPW ? G.nblocks - g0 : Slab<N>::BPW);
}

// Loads the 1D factor table into registers.  FP64 tables go through LDS so
// that they land in VGPRs; FP32 tables are read with wave-uniform addresses
// and stay in scalar registers.
template <typename TC, int COUNT>
__device__ __forceinline__ void load_table(TC (&dst)[COUNT], const TC* __restrict__ tab, TC* stab) {
    if constexpr (sizeof(TC) == 8) {
        for (int e = threadIdx.x; e < COUNT; e += 64) stab[e] = tab[e];
        wave_sync();
#pragma unroll
        for (int i = 0; i < COUNT; ++i) dst[i] = stab[i];
    } else {
#pragma unroll
        for (int i = 0; i < COUNT; ++i) dst[i] = tab[i];
    }
}

// Stages COUNT table entries in LDS (stab) for reads from there.
template <typename TC, int COUNT>
__device__ __forceinline__ void stage_table(const TC* __restrict__ tab, TC* stab) {
    for (int e = threadIdx.x; e < COUNT; e += 64) stab[e] = tab[e];
    wave_sync();
}

// ------------------------------------------------------------ tile bodies
// Each body handles one tile with the lane's pencil coordinates pc and the
// per-block scalings (sx, sy, sz); it starts with the lane's z-pencil in
// registers and synchronises the wave between phases.

// v = A x (global output).  A1, A2: the lane's LDS scratch slabs.
template <int N, typename TS, typename TC>
__device__ __forceinline__ void eo_apply_body(const Pencil<N>& pc, const TC (&x)[N], TS* __restrict__ v,
                                              const GArgs& G, int64_t g0, TC* A1, TC* A2, const TC* ME,
                                              const TC* MO, const TC* PE, const TC* PO, TC sx, TC sy, TC sz) {
    using L = Slab<N>;
    constexpr int HC = EOShape<N>::HC, H = EOShape<N>::H;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {  // z: lane (i, j); t = M x, w = P x
        TC e[HC], o[H], E[HC], O[H], y[N];
        eo_split<N>(x, e, o);
        eo_mul<N>(ME, MO, e, o, E, O);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int k = 0; k < N; ++k) A1[L::at(pa, pb, k)] = y[k];
        eo_mul<N>(PE, PO, e, o, E, O);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int k = 0; k < N; ++k) A2[L::at(pa, pb, k)] = y[k];
    }
    wave_sync();
    if (pc.act) {  // y: lane (i, k); a = s_x M t, b = s_y P t + s_z M w
        TC et[HC], ot[H], ew[HC], ow[H], E[HC], O[H], E2[HC], O2[H], y[N];
#pragma unroll
        for (int j = 0; j < N; ++j) y[j] = A1[L::at(pa, j, pb)];
        eo_split<N>(y, et, ot);
#pragma unroll
        for (int j = 0; j < N; ++j) y[j] = A2[L::at(pa, j, pb)];
        eo_split<N>(y, ew, ow);
        eo_mul<N>(ME, MO, et, ot, E, O);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int j = 0; j < N; ++j) A1[L::at(pa, j, pb)] = y[j] * sx;
        eo_mul<N>(PE, PO, et, ot, E, O);
        eo_mul<N>(ME, MO, ew, ow, E2, O2);
#pragma unroll
        for (int i = 0; i < HC; ++i) E[i] = fma(sy, E[i], sz * E2[i]);
#pragma unroll
        for (int i = 0; i < H; ++i) O[i] = fma(sy, O[i], sz * O2[i]);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int j = 0; j < N; ++j) A2[L::at(pa, j, pb)] = y[j];
    }
    wave_sync();
    if (pc.act) {  // x: lane (j, k); v = P a + M b, stored to global
        TC y[N], ea[HC], oa[H], eb[HC], ob[H], E[HC], O[H], E2[HC], O2[H];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = A1[L::at(i, pa, pb)];
        eo_split<N>(y, ea, oa);
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = A2[L::at(i, pa, pb)];
        eo_split<N>(y, eb, ob);
        eo_mul<N>(PE, PO, ea, oa, E, O);
        eo_mul<N>(ME, MO, eb, ob, E2, O2);
#pragma unroll
        for (int i = 0; i < HC; ++i) E[i] += E2[i];
#pragma unroll
        for (int i = 0; i < H; ++i) O[i] += O2[i];
        eo_join<N>(E, O, y);
        TS* out = v + G.offset + block_base(g0 + pc.w, G.logB, L::N3);
        // a wave's store covers whole 128-byte lines only when an x-plane
        // does; only then does the streaming hint not split lines
        constexpr bool kWholeLines = (N * N * sizeof(TS)) % 128 == 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            TS* o = out + (static_cast<int64_t>((i * N + pa) * N + pb) << G.logB);
            if constexpr (kWholeLines) stg(o, y[i]);
            else stc(o, y[i]);
        }
    }
    wave_sync();
}

// The three middle phases of D^{-1} on the lane's slab A1, which on entry
// holds S_z^T applied along z; on exit A1 holds S_y S_x Lambda^{-1} ... along
// every axis but z (backward z is left to the caller).
template <int N, typename TC>
__device__ __forceinline__ void eo_inverse_mid(const Pencil<N>& pc, TC* A1, const TC* SE, const TC* SO,
                                               const TC* lam, TC sx, TC sy, TC sz) {
    using L = Slab<N>;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {  // y forward: lane (i, c)
        TC a[N], y[N];
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = A1[L::at(pa, j, pb)];
        eo_fwd<N>(SE, SO, a, y);
#pragma unroll
        for (int b = 0; b < N; ++b) A1[L::at(pa, b, pb)] = y[b];
    }
    wave_sync();
    if (pc.act) {  // x forward, scale, x backward: lane (b, c)
        TC a[N], y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) a[i] = A1[L::at(i, pa, pb)];
        eo_fwd<N>(SE, SO, a, y);
        const TC mu_bc = lam[pa] * sy + lam[pb] * sz;
#pragma unroll
        for (int c = 0; c < N; ++c) y[c] *= recip(fma(lam[c], sx, mu_bc));
        eo_bwd<N>(SE, SO, y, a);
#pragma unroll
        for (int i = 0; i < N; ++i) A1[L::at(i, pa, pb)] = a[i];
    }
    wave_sync();
    if (pc.act) {  // y backward: lane (i, c)
        TC y[N], a[N];
#pragma unroll
        for (int b = 0; b < N; ++b) y[b] = A1[L::at(pa, b, pb)];
        eo_bwd<N>(SE, SO, y, a);
#pragma unroll
        for (int j = 0; j < N; ++j) A1[L::at(pa, j, pb)] = a[j];
    }
    wave_sync();
}

// x = D^{-1} r for one tile: r's z-pencil in registers, the result stored
// to global memory from x-pencils.  The 1D transforms along different axes
// commute, so the phases run z, x forward, then y forward + scaling + y
// backward, then z and x backward: the last phase is along x, whose lanes
// (j, k) write consecutive addresses of an x-plane (whole 128-byte lines for
// n = 8 at every storage type and n = 4 in FP64), like the apply's output.
template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void eo_inverse_body(const Pencil<N>& pc, const TC (&r)[N], TS* __restrict__ x,
                                                const GArgs& G, int64_t g0, TC* A1, const TC* SE, const TC* SO,
                                                const TC* lam, TC sx, TC sy, TC sz) {
    using L = Slab<N>;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {  // z forward: lane (i, j)
        TC y[N];
        eo_fwd<N>(SE, SO, r, y);
#pragma unroll
        for (int c = 0; c < N; ++c) A1[L::at(pa, pb, c)] = y[c];
    }
    wave_sync();
    if (pc.act) {  // x forward: lane (j, c)
        TC a[N], y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) a[i] = A1[L::at(i, pa, pb)];
        eo_fwd<N>(SE, SO, a, y);
#pragma unroll
        for (int i = 0; i < N; ++i) A1[L::at(i, pa, pb)] = y[i];
    }
    wave_sync();
    if (pc.act) {  // y forward, scaling, y backward: lane (a, c)
        TC a[N], y[N];
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = A1[L::at(pa, j, pb)];
        eo_fwd<N>(SE, SO, a, y);
        const TC mu_ac = lam[pa] * sx + lam[pb] * sz;
#pragma unroll
        for (int b = 0; b < N; ++b) y[b] *= recip(fma(lam[b], sy, mu_ac));
        eo_bwd<N>(SE, SO, y, a);
#pragma unroll
        for (int j = 0; j < N; ++j) A1[L::at(pa, j, pb)] = a[j];
    }
    wave_sync();
    if (pc.act) {  // z backward: lane (a, j)
        TC y[N], a[N];
#pragma unroll
        for (int c = 0; c < N; ++c) y[c] = A1[L::at(pa, pb, c)];
        eo_bwd<N>(SE, SO, y, a);
#pragma unroll
        for (int k = 0; k < N; ++k) A1[L::at(pa, pb, k)] = a[k];
    }
    wave_sync();
    if (pc.act) {  // x backward: lane (j, k), x-plane rows stored to global memory
        TC y[N], a[N];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = A1[L::at(i, pa, pb)];
        eo_bwd<N>(SE, SO, y, a);
        TS* out = x + G.offset + block_base(g0 + pc.w, G.logB, L::N3);
        constexpr bool kWholeLines = (N * N * sizeof(TS)) % 128 == 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            TS* o = out + (static_cast<int64_t>((i * N + pa) * N + pb) << G.logB);
            if constexpr (kWholeLines) stg(o, a[i]);
            else stc(o, a[i]);
        }
    }
    wave_sync();
}

// dst = A x with the lane's z-pencil of x in registers, through LDS (dst
// may alias t1); t1, t2 scratch slabs.  dst receives the product in slab
// layout, written by x-pencils; the wave is synchronised on return.
template <int N, typename TC>
__device__ __forceinline__ void eo_apply_regs(const Pencil<N>& pc, const TC (&x)[N], TC* dst, TC* t1, TC* t2,
                                              const TC* ME, const TC* MO, const TC* PE, const TC* PO, TC sx, TC sy,
                                              TC sz) {
    using L = Slab<N>;
    constexpr int HC = EOShape<N>::HC, H = EOShape<N>::H;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {
        TC e[HC], o[H], E[HC], O[H], y[N];
        eo_split<N>(x, e, o);
        eo_mul<N>(ME, MO, e, o, E, O);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int k = 0; k < N; ++k) t1[L::at(pa, pb, k)] = y[k];
        eo_mul<N>(PE, PO, e, o, E, O);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int k = 0; k < N; ++k) t2[L::at(pa, pb, k)] = y[k];
    }
    wave_sync();
    if (pc.act) {
        TC et[HC], ot[H], ew[HC], ow[H], E[HC], O[H], E2[HC], O2[H], y[N];
#pragma unroll
        for (int j = 0; j < N; ++j) y[j] = t1[L::at(pa, j, pb)];
        eo_split<N>(y, et, ot);
#pragma unroll
        for (int j = 0; j < N; ++j) y[j] = t2[L::at(pa, j, pb)];
        eo_split<N>(y, ew, ow);
        eo_mul<N>(ME, MO, et, ot, E, O);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int j = 0; j < N; ++j) t1[L::at(pa, j, pb)] = y[j] * sx;
        eo_mul<N>(PE, PO, et, ot, E, O);
        eo_mul<N>(ME, MO, ew, ow, E2, O2);
#pragma unroll
        for (int i = 0; i < HC; ++i) E[i] = fma(sy, E[i], sz * E2[i]);
#pragma unroll
        for (int i = 0; i < H; ++i) O[i] = fma(sy, O[i], sz * O2[i]);
        eo_join<N>(E, O, y);
#pragma unroll
        for (int j = 0; j < N; ++j) t2[L::at(pa, j, pb)] = y[j];
    }
    wave_sync();
    if (pc.act) {
        TC y[N], ea[HC], oa[H], eb[HC], ob[H], E[HC], O[H], E2[HC], O2[H];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = t1[L::at(i, pa, pb)];
        eo_split<N>(y, ea, oa);
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = t2[L::at(i, pa, pb)];
        eo_split<N>(y, eb, ob);
        eo_mul<N>(PE, PO, ea, oa, E, O);
        eo_mul<N>(ME, MO, eb, ob, E2, O2);
#pragma unroll
        for (int i = 0; i < HC; ++i) E[i] += E2[i];
#pragma unroll
        for (int i = 0; i < H; ++i) O[i] += O2[i];
        eo_join<N>(E, O, y);
#pragma unroll
        for (int i = 0; i < N; ++i) dst[L::at(i, pa, pb)] = y[i];
    }
    wave_sync();
}

// dst = A src entirely in LDS (dst may alias src); t1, t2 scratch slabs.
template <int N, typename TC>
__device__ __forceinline__ void eo_apply_lds(const Pencil<N>& pc, const TC* src, TC* dst, TC* t1, TC* t2,
                                             const TC* ME, const TC* MO, const TC* PE, const TC* PO, TC sx, TC sy,
                                             TC sz) {
    using L = Slab<N>;
    TC x[N];
    if (pc.act)
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = src[L::at(pc.pa, pc.pb, k)];
    eo_apply_regs<N, TC>(pc, x, dst, t1, t2, ME, MO, PE, PO, sx, sy, sz);
}

// r <- D^{-1} r with the lane's z-pencil of r in registers on entry and on
// return, through the LDS slab (each phase updates its own pencils).
template <int N, typename TC>
__device__ __forceinline__ void eo_inverse_regs(const Pencil<N>& pc, TC (&r)[N], TC* slab, const TC* SE,
                                                const TC* SO, const TC* lam, TC sx, TC sy, TC sz) {
    using L = Slab<N>;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {
        TC y[N];
        eo_fwd<N>(SE, SO, r, y);
#pragma unroll
        for (int c = 0; c < N; ++c) slab[L::at(pa, pb, c)] = y[c];
    }
    wave_sync();
    eo_inverse_mid<N>(pc, slab, SE, SO, lam, sx, sy, sz);
    if (pc.act) {
        TC y[N];
#pragma unroll
        for (int c = 0; c < N; ++c) y[c] = slab[L::at(pa, pb, c)];
        eo_bwd<N>(SE, SO, y, r);
    }
    wave_sync();
}

// slab <- D^{-1} slab entirely in LDS (each phase updates its own pencils).
template <int N, typename TC>
__device__ __forceinline__ void eo_inverse_lds(const Pencil<N>& pc, TC* slab, const TC* SE, const TC* SO,
                                               const TC* lam, TC sx, TC sy, TC sz) {
    using L = Slab<N>;
    TC a[N];
    if (pc.act)
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = slab[L::at(pc.pa, pc.pb, k)];
    eo_inverse_regs<N, TC>(pc, a, slab, SE, SO, lam, sx, sy, sz);
    if (pc.act)
#pragma unroll
        for (int k = 0; k < N; ++k) slab[L::at(pc.pa, pc.pb, k)] = a[k];
    wave_sync();
}

// ------------------------------------------------------------ solve tile
// LDS workspace of one solve tile: the iterate x and two scratch slabs; the
// product lands in t1 and the scaled residual (in the inner precision) in
// t2, so the whole tile needs three slabs.
template <int N, typename TI>
struct SolveLds {
    static constexpr int SZ = Slab<N>::BPW * Slab<N>::size;
    static_assert(sizeof(TI) <= sizeof(double), "inner type wider than the slab");
    double xs[SZ], t1[SZ], t2[SZ];
    double part[2][64];
    double red[3][Slab<N>::BPW];
    int done[Slab<N>::BPW];
};

// Block-local iterative refinement of one tile (a wave, BPW blocks), with
// the block operator and the inner inverse given as callables on the LDS
// slabs (apply_lds(pc, src, dst, t1, t2) in FP64 with dst allowed to be t1,
// inverse_lds(pc, slab) in TI, both for the lane's pencil pc):
//   r = b - D x (FP64), s = ||r||_inf, d = D~^{-1} (r / s) in precision TI
//   (input and output rounded to FP16 / BF16 for RND),
//   x <- x + s d (FP64), until ||r||_2 <= rtol ||b||_2 or maxit corrections.
// x stays in LDS for all iterations (read once, written once); each lane
// reads its z-pencil of b for every residual (from cache after the first);
// per-block norms are reduced over the block's pencils through LDS.
template <int N, typename TI, int RND, typename ApplyF, typename InvF>
__device__ __forceinline__ void solve_tile(const double* __restrict__ b, double* __restrict__ x, const GArgs& G,
                                           int64_t g0, int nvalid, SolveLds<N, TI>& S, ApplyF apply_lds,
                                           InvF inverse_lds, double rtol, int maxit, int32_t* __restrict__ iters,
                                           double* __restrict__ relres, int64_t block0, SolveAcc& acc) {
    using L = Slab<N>;
    bool nz = false;
    for (int e = threadIdx.x; e < nvalid * L::N3; e += 64) {
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        const double xv = x[G.offset + block_base(g0 + w, G.logB, L::N3) + (static_cast<int64_t>(q) << G.logB)];
        S.xs[w * L::size + L::lin(q)] = xv;
        nz = nz || xv != 0.0;
    }
    // the residual of an all-zero x is b: the first product is skipped
    // when every x of the tile is zero on entry
    bool need_apply = __any(nz);
    const Pencil<N> pc(nvalid);
    const int lane = threadIdx.x;
    const int so = (pc.w < L::BPW ? pc.w : 0) * L::size;
    TI* rs = reinterpret_cast<TI*>(S.t2) + so;
    const double* bpen = pc.act ? pencil_ptr<N>(b, G, g0 + pc.w, pc.pa, pc.pb) : b;
    double bsq = 0.0;
    if (pc.act) {
        double bp[N];
        pencil_load<N, false>(bp, bpen, G.logB);
#pragma unroll
        for (int k = 0; k < N; ++k) bsq = fma(bp[k], bp[k], bsq);
    }
    S.part[0][lane] = bsq;
    wave_sync();
    if (pc.act && pc.pa == 0 && pc.pb == 0) {
        double sacc = 0.0;
        for (int l = 0; l < L::N2; ++l) sacc += S.part[0][lane + l];
        S.red[0][pc.w] = sacc;
        S.done[pc.w] = 0;
    }
    wave_sync();
    int it = 0;
    const double bn = pc.act ? S.red[0][pc.w] : 0.0;
    double rel = 0.0;
    if (pc.act && bn == 0.0)
        for (int k = 0; k < N; ++k) S.xs[so + L::at(pc.pa, pc.pb, k)] = 0.0;
    for (;;) {
        if (need_apply) apply_lds(pc, S.xs + so, S.t1 + so, S.t1 + so, S.t2 + so);
        double rr = 0.0, rmax = 0.0;
        if (pc.act) {  // the residual overwrites the product in t1; b is re-read (cached)
            double bp[N];
            pencil_load<N, false>(bp, bpen, G.logB);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int a = so + L::at(pc.pa, pc.pb, k);
                const double rv = need_apply ? bp[k] - S.t1[a] : bp[k];
                S.t1[a] = rv;
                rr = fma(rv, rv, rr);
                rmax = fmax(rmax, fabs(rv));
            }
        }
        S.part[0][lane] = rr;
        S.part[1][lane] = rmax;
        wave_sync();
        if (pc.act && pc.pa == 0 && pc.pb == 0) {
            double s2 = 0.0, m = 0.0;
            for (int l = 0; l < L::N2; ++l) {
                s2 += S.part[0][lane + l];
                m = fmax(m, S.part[1][lane + l]);
            }
            S.red[1][pc.w] = s2;
            S.red[2][pc.w] = m;
        }
        wave_sync();
        bool mine_done = true;
        if (pc.act && !S.done[pc.w]) {
            rel = bn == 0.0 ? 0.0 : sqrt(S.red[1][pc.w] / bn);
            mine_done = !(rel > rtol) || it >= maxit;
        }
        wave_sync();
        if (pc.act && pc.pa == 0 && pc.pb == 0 && mine_done) S.done[pc.w] = 1;
        if (!__any(pc.act && !mine_done)) break;
        const double rmax_b = pc.act ? S.red[2][pc.w] : 0.0;
        const double inv_s = (pc.act && !mine_done && rmax_b > 0.0) ? 1.0 / rmax_b : 0.0;
        if (pc.act)
#pragma unroll
            for (int k = 0; k < N; ++k)
                rs[L::at(pc.pa, pc.pb, k)] =
                    round_to<RND>(static_cast<TI>(S.t1[so + L::at(pc.pa, pc.pb, k)] * inv_s));
        wave_sync();
        inverse_lds(pc, rs);
        if (pc.act && !mine_done) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int a = so + L::at(pc.pa, pc.pb, k);
                S.xs[a] = fma(rmax_b, static_cast<double>(round_to<RND>(rs[L::at(pc.pa, pc.pb, k)])), S.xs[a]);
            }
            ++it;
        }
        need_apply = true;
        wave_sync();
    }
    for (int e = threadIdx.x; e < nvalid * L::N3; e += 64) {
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        x[G.offset + block_base(g0 + w, G.logB, L::N3) + (static_cast<int64_t>(q) << G.logB)] =
            S.xs[w * L::size + L::lin(q)];
    }
    if (pc.act && pc.pa == 0 && pc.pb == 0) {
        const int64_t gidx = block0 + g0 + pc.w;
        if (iters) iters[gidx] = it;
        if (relres) relres[gidx] = rel;
        acc.add(it, rel, rtol);
    }
    wave_sync();
}

// Sum and maximum over the wave by an xor butterfly: every lane ends with
// the same value, bit for bit (each step adds or compares the same pair).
__device__ __forceinline__ double wave_allsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_allmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// LDS workspace of the register-resident solve tile: two FP64 scratch
// slabs for the product (the first also holds the inner solve's slab, in
// the inner precision) and the per-block reductions.
template <int N>
struct SolveLdsR {
    static constexpr int SZ = Slab<N>::BPW * Slab<N>::size;
    double t1[SZ], t2[SZ];
    double part[2][64];
    double red[3][Slab<N>::BPW];
    int done[Slab<N>::BPW];
};

// Block-local iterative refinement of one tile with the iterate, the
// right-hand side and the residual in registers: each active lane owns the
// z-pencil (pa, pb) of its block w of x and b (read once from memory, x
// written once), the product A x goes through the two LDS slabs
// (apply_regs(pc, xr, dst, t1, t2), ending in slab layout in t1) and the
// inner inverse takes and returns the lane's pencil in registers
// (inverse_regs(pc, d, slab) in precision TI).  Per correction:
//   r = b - D x (FP64), s = ||r||_inf, d = D~^{-1} (r / s) in TI (input and
//   output rounded to FP16 / BF16 for RND), x <- x + s d (FP64),
// until ||r||_2 <= rtol ||b||_2 or maxit corrections.  Per-block norms are
// reduced over the block's pencils through LDS.
template <int N, typename TI, int RND, bool VP, typename ApplyF, typename InvF>
__device__ __forceinline__ void solve_tile_reg(const double* __restrict__ b, double* __restrict__ x,
                                               const GArgs& G, int64_t g0, int nvalid, SolveLdsR<N>& S,
                                               ApplyF apply_regs, InvF inverse_regs, double rtol, int maxit,
                                               int32_t* __restrict__ iters, double* __restrict__ relres,
                                               int64_t block0, SolveAcc& acc) {
    using L = Slab<N>;
    const Pencil<N> pc(nvalid);
    const int lane = threadIdx.x;
    const int so = (pc.w < L::BPW ? pc.w : 0) * L::size;
    double xr[N], br[N];
    bool nz = false;
    double bsq = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) xr[k] = br[k] = 0.0;
    if (pc.act) {
        pencil_load<N, VP>(xr, pencil_ptr<N>(static_cast<const double*>(x), G, g0 + pc.w, pc.pa, pc.pb), G.logB);
        pencil_load<N, VP>(br, pencil_ptr<N>(b, G, g0 + pc.w, pc.pa, pc.pb), G.logB);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            nz = nz || xr[k] != 0.0;
            bsq = fma(br[k], br[k], bsq);
        }
    }
    // the residual of an all-zero x is b: the first product is skipped
    // when every x of the tile is zero on entry
    bool need_apply = __any(nz);
    // per-block sums: over the whole wave when the tile is one block (n >= 6),
    // else over the block's lanes through LDS
    constexpr bool kOne = L::BPW == 1;
    double bn;
    if constexpr (kOne) {
        bn = wave_allsum(bsq);
    } else {
        S.part[0][lane] = bsq;
        wave_sync();
        if (pc.act && pc.pa == 0 && pc.pb == 0) {
            double sacc = 0.0;
            for (int l = 0; l < L::N2; ++l) sacc += S.part[0][lane + l];
            S.red[0][pc.w] = sacc;
            S.done[pc.w] = 0;
        }
        wave_sync();
        bn = pc.act ? S.red[0][pc.w] : 0.0;
    }
    bool done_before = false;   // (one-block tiles) the block met its test in an earlier pass
    int it = 0;
    double rel = 0.0;
    if (pc.act && bn == 0.0)
#pragma unroll
        for (int k = 0; k < N; ++k) xr[k] = 0.0;
    for (;;) {
        double r[N];
        if (need_apply) {
            apply_regs(pc, xr, S.t1 + so, S.t1 + so, S.t2 + so);
#pragma unroll
            for (int k = 0; k < N; ++k) r[k] = pc.act ? br[k] - S.t1[so + L::at(pc.pa, pc.pb, k)] : 0.0;
        } else {
#pragma unroll
            for (int k = 0; k < N; ++k) r[k] = br[k];
        }
        double rr = 0.0, rmax = 0.0;
        if (pc.act)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                rr = fma(r[k], r[k], rr);
                rmax = fmax(rmax, fabs(r[k]));
            }
        double rsq_b, rmax_b;
        bool mine_done = true;
        if constexpr (kOne) {
            rsq_b = wave_allsum(rr);
            rmax_b = wave_allmax(rmax);
            if (!done_before) {
                rel = bn == 0.0 ? 0.0 : sqrt(rsq_b / bn);
                mine_done = !(rel > rtol) || it >= maxit;
            }
            done_before = mine_done;
            if (mine_done) break;   // wave-uniform: the tile is one block
        } else {
            S.part[0][lane] = rr;
            S.part[1][lane] = rmax;
            wave_sync();
            if (pc.act && pc.pa == 0 && pc.pb == 0) {
                double s2 = 0.0, m = 0.0;
                for (int l = 0; l < L::N2; ++l) {
                    s2 += S.part[0][lane + l];
                    m = fmax(m, S.part[1][lane + l]);
                }
                S.red[1][pc.w] = s2;
                S.red[2][pc.w] = m;
            }
            wave_sync();
            if (pc.act && !S.done[pc.w]) {
                rel = bn == 0.0 ? 0.0 : sqrt(S.red[1][pc.w] / bn);
                mine_done = !(rel > rtol) || it >= maxit;
            }
            wave_sync();
            if (pc.act && pc.pa == 0 && pc.pb == 0 && mine_done) S.done[pc.w] = 1;
            if (!__any(pc.act && !mine_done)) break;
            rmax_b = pc.act ? S.red[2][pc.w] : 0.0;
        }
        (void)rsq_b;
        const double inv_s = (pc.act && !mine_done && rmax_b > 0.0) ? 1.0 / rmax_b : 0.0;
        TI d[N];
#pragma unroll
        for (int k = 0; k < N; ++k) d[k] = round_to<RND>(static_cast<TI>(r[k] * inv_s));
        inverse_regs(pc, d, reinterpret_cast<TI*>(S.t1) + so);
        if (pc.act && !mine_done) {
#pragma unroll
            for (int k = 0; k < N; ++k) xr[k] = fma(rmax_b, static_cast<double>(round_to<RND>(d[k])), xr[k]);
            ++it;
        }
        need_apply = true;
    }
    if (pc.act) pencil_store<N, VP>(const_cast<double*>(pencil_ptr<N>(x, G, g0 + pc.w, pc.pa, pc.pb)), xr, G.logB);
    if (pc.act && pc.pa == 0 && pc.pb == 0) {
        const int64_t gidx = block0 + g0 + pc.w;
        if (iters) iters[gidx] = it;
        if (relres) relres[gidx] = rel;
        acc.add(it, rel, rtol);
    }
    wave_sync();
}

// Factor tables of a tile kernel, in registers.  FP64 tables go through LDS
// so that they land in VGPRs; FP32 tables use wave-uniform loads (SGPRs).
template <int N, typename TC>
struct ApplyTab {
    static constexpr int COUNT = 2 * (EOShape<N>::SE + EOShape<N>::SO);
    TC v[COUNT];
    __device__ __forceinline__ const TC* ME() const { return v; }
    __device__ __forceinline__ const TC* MO() const { return v + EOShape<N>::SE; }
    __device__ __forceinline__ const TC* PE() const { return v + EOShape<N>::SE + EOShape<N>::SO; }
    __device__ __forceinline__ const TC* PO() const { return v + 2 * EOShape<N>::SE + EOShape<N>::SO; }
};
template <int N, typename TC>
struct InvTab {
    static constexpr int COUNT = EOShape<N>::SE + EOShape<N>::SO;
    TC v[COUNT];
    __device__ __forceinline__ const TC* SE() const { return v; }
    __device__ __forceinline__ const TC* SO() const { return v + EOShape<N>::SE; }
};

// The solve tile with the even-odd reference operators: per-block scalings
// from the edge lengths, iterate and residual in registers
// (solve_tile_reg).  tA: the apply table ME|MO|PE|PO (FP64), tS: the inverse
// table SE|SO (TI), lam: the eigenvalues (TI); each may point to registers
// or to LDS.
template <int N, typename TI, int RND, bool VP>
__device__ __forceinline__ void eo_solve_tile(const double* __restrict__ b, double* __restrict__ x, const GArgs& G,
                                              int64_t g0, int nvalid, SolveLdsR<N>& S, const double* tA,
                                              const TI* tS, const TI* lam, double rtol, int maxit,
                                              int32_t* __restrict__ iters, double* __restrict__ relres,
                                              int64_t block0, SolveAcc& acc) {
    using E = EOShape<N>;
    const Pencil<N> pc(nvalid);
    double sx = 1.0, sy = 1.0, sz = 1.0;
    if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
    const TI sxi = static_cast<TI>(sx), syi = static_cast<TI>(sy), szi = static_cast<TI>(sz);
    solve_tile_reg<N, TI, RND, VP>(
        b, x, G, g0, nvalid, S,
        [&](const Pencil<N>& p, const double (&xr)[N], double* dst, double* t1, double* t2) {
            eo_apply_regs<N, double>(p, xr, dst, t1, t2, tA, tA + E::SE, tA + E::SE + E::SO, tA + 2 * E::SE + E::SO,
                                     sx, sy, sz);
        },
        [&](const Pencil<N>& p, TI (&d)[N], TI* slab) {
            eo_inverse_regs<N, TI>(p, d, slab, tS, tS + E::SE, lam, sxi, syi, szi);
        },
        rtol, maxit, iters, relres, block0, acc);
}

// Copies `count` table entries to LDS (always: the eigenvalues are indexed
// per lane) and into the register array; stab must hold count entries.
// VREG selects the vector-register copy (default: for 8-byte entries).
template <typename TC, int COUNT, bool VREG = (sizeof(TC) == 8)>
__device__ __forceinline__ void table_to_regs(TC (&dst)[COUNT], const TC* __restrict__ tab, TC* stab, int count) {
    wave_sync();
    for (int e = threadIdx.x; e < count; e += 64) stab[e] = tab[e];
    wave_sync();
    if constexpr (VREG) {
#pragma unroll
        for (int i = 0; i < COUNT; ++i) dst[i] = stab[i];
    } else {
#pragma unroll
        for (int i = 0; i < COUNT; ++i) dst[i] = tab[i];
    }
}

}  // namespace tpfdm
