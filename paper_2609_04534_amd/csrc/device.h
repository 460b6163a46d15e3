// Device-side helpers shared by the kernel translation units: storage
// conversions, kernel parameter blocks, block addressing and reciprocals.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tpfdm {

// ------------------------------------------------------------ storage types
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// float -> bfloat16 with round-to-nearest-even (add half an ulp of the
// truncated format plus the tie bit, then truncate); NaN stays quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

template <typename TC> __device__ __forceinline__ TC ldc(const double* p) { return static_cast<TC>(*p); }
template <typename TC> __device__ __forceinline__ TC ldc(const float* p) { return static_cast<TC>(*p); }
template <typename TC> __device__ __forceinline__ TC ldc(const _Float16* p) {
    return static_cast<TC>(static_cast<float>(*p));
}
template <typename TC> __device__ __forceinline__ TC ldc(const bf16_t* p) {
    return static_cast<TC>(bf16_to_f32(p->bits));
}
__device__ __forceinline__ void stc(double* p, double v) { *p = v; }
__device__ __forceinline__ void stc(float* p, float v) { *p = v; }
__device__ __forceinline__ void stc(_Float16* p, float v) { *p = static_cast<_Float16>(v); }
__device__ __forceinline__ void stc(bf16_t* p, float v) { p->bits = f32_to_bf16(v); }

// ------------------------------------------------------------ kernel params
template <int N, typename T>
struct Pair {      // reference mass M and operator P (K or A_hat), row-major
    T m[N * N];
    T p[N * N];
};
template <int N, typename T>
struct Eig {       // reference eigenvectors S (column j = vector j) and eigenvalues
    T s[N * N];
    T lam[N];
};

struct GArgs {
    const double* h;
    int64_t nblocks;
    int64_t offset;
    int logB;
};

// Element offset of block g's DoF 0 inside its group; DoF q sits at
// base + (q << logB).
__device__ __forceinline__ int64_t block_base(int64_t g, int logB, int n3) {
    return (((g >> logB) * n3) << logB) + (g & ((int64_t(1) << logB) - 1));
}

template <typename TC>
__device__ __forceinline__ void block_scales(const double* h, int64_t g, TC& sx, TC& sy, TC& sz) {
    const double hx = h[3 * g], hy = h[3 * g + 1], hz = h[3 * g + 2];
    sx = static_cast<TC>(hy * hz / hx);
    sy = static_cast<TC>(hx * hz / hy);
    sz = static_cast<TC>(hx * hy / hz);
}

// Reciprocal: hardware estimate refined by Newton-Raphson steps
// r <- r + r (1 - a r), each of which roughly doubles the correct bits.
__device__ __forceinline__ double recip(double a) {
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float a) {
    float r = __builtin_amdgcn_rcpf(a);
    float e = fmaf(-a, r, 1.0f);
    return fmaf(r, e, r);
}

// Synchronises the lanes of one wave around an LDS exchange.  Every kernel
// that uses it runs one wave per workgroup; a wave's LDS instructions execute
// in program order, so only the compiler must be kept from moving LDS
// accesses across this point.  Wavefront-scope fences do that without the
// global-memory wait of a workgroup barrier, which would drain the loads a
// kernel has in flight for its next tiles.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ wave tiles
// A workgroup of one wave owns BPW = max(1, 64 / n^2) consecutive blocks.
// Lane l works on block w = l / n^2 of the tile and on pencil l % n^2 of it.
// Each block's n^3 slab sits in LDS, element (i, j, k) at (i n + j)(n+1) + k;
// the pad of one element per pencil spreads strided pencil reads over banks.
template <int N>
struct Slab {
    static constexpr int N2 = N * N;
    static constexpr int N3 = N * N * N;
    static constexpr int BPW = N2 >= 64 ? 1 : 64 / N2;
    static constexpr int size = N * N * (N + 1);
    __device__ static __forceinline__ int at(int i, int j, int k) { return (i * N + j) * (N + 1) + k; }
    __device__ static __forceinline__ int lin(int e) { return e + e / N; }
};

// Per-lane pencil coordinates inside the tile.
template <int N>
struct Pencil {
    int w;       // block within the tile
    int pa, pb;  // pencil coordinates (meaning depends on the phase)
    bool act;    // lane owns a pencil of an existing block
    __device__ __forceinline__ Pencil(int nvalid) {
        const int lane = threadIdx.x;
        w = lane / Slab<N>::N2;
        const int p = lane - w * Slab<N>::N2;
        pa = p / N;
        pb = p - pa * N;
        act = w < Slab<N>::BPW && w < nvalid;
    }
};

}  // namespace tpfdm
