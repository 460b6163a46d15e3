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

// float -> bfloat16, round to nearest even (gfx950 converts in hardware,
// v_cvt_pk_bf16_f32; NaN stays NaN).  Branch-free: a per-element branch
// around the NaN case would serialise the stores that follow it.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
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

// Streaming accesses to the caller's vectors.  Every element of an input is
// read once and every element of an output written once per call, so these
// carry the nontemporal hint: the lines are not kept in the caches for reuse
// that never comes (measured: +10-16 % HBM throughput on the n = 4 kernels).
// Only for access patterns where each wave instruction covers whole 128-byte
// lines: a line fetched in pieces by several instructions must stay cached
// between them, and with the hint it is fetched again (measured: -20 % on
// the n = 8 pencil loads).
template <typename TC> __device__ __forceinline__ TC ldg(const double* p) {
    return static_cast<TC>(__builtin_nontemporal_load(p));
}
template <typename TC> __device__ __forceinline__ TC ldg(const float* p) {
    return static_cast<TC>(__builtin_nontemporal_load(p));
}
template <typename TC> __device__ __forceinline__ TC ldg(const _Float16* p) {
    return static_cast<TC>(static_cast<float>(__builtin_nontemporal_load(p)));
}
template <typename TC> __device__ __forceinline__ TC ldg(const bf16_t* p) {
    return static_cast<TC>(bf16_to_f32(__builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p))));
}
__device__ __forceinline__ void stg(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void stg(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void stg(_Float16* p, float v) { __builtin_nontemporal_store(static_cast<_Float16>(v), p); }
__device__ __forceinline__ void stg(bf16_t* p, float v) {
    __builtin_nontemporal_store(f32_to_bf16(v), reinterpret_cast<uint16_t*>(p));
}
// Rounding of an FP32 value to the precision of a low-precision inner solve
// (RND: 0 none, 1 FP16, 2 BF16), round to nearest even.
enum { RND_NONE = 0, RND_F16 = 1, RND_BF16 = 2 };
template <int RND, typename T> __device__ __forceinline__ T round_to(T v) {
    if constexpr (RND == RND_F16) return static_cast<T>(static_cast<float>(static_cast<_Float16>(static_cast<float>(v))));
    else if constexpr (RND == RND_BF16) return static_cast<T>(bf16_to_f32(f32_to_bf16(static_cast<float>(v))));
    else return v;
}

// Streaming (NT) or plain access, chosen at compile time.
template <bool NT, typename TC, typename TS> __device__ __forceinline__ TC ldv(const TS* p) {
    if constexpr (NT) return ldg<TC>(p);
    else return ldc<TC>(p);
}
template <bool NT, typename TS, typename TC> __device__ __forceinline__ void stv(TS* p, TC v) {
    if constexpr (NT) stg(p, v);
    else stc(p, v);
}
// A lane-per-block wave moves one element of 64 consecutive blocks per
// instruction: whole lines when B * sizeof(element) >= 128 bytes.
template <typename TS> inline bool lane_whole_lines(int logB) {
    return (static_cast<int64_t>(sizeof(TS)) << logB) >= 128;
}


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
__host__ __device__ __forceinline__ int64_t block_base(int64_t g, int logB, int n3) {
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

// Per-lane accumulation of block results; flush() reduces over the wave and
// lane 0 stores the workgroup's partial summary (no atomics: a solve over
// millions of blocks would otherwise serialise on one summary address).
struct SolveAcc {
    int max_iters = 0;
    int n_failed = 0;
    int nonfinite = 0;
    double max_relres = 0.0;
    __device__ __forceinline__ void add(int it, double rel, double rtol) {
        max_iters = it > max_iters ? it : max_iters;
        const bool finite = (rel == rel) && rel <= 1.7976931348623157e308;
        if (!(rel <= rtol)) ++n_failed;
        if (!finite) ++nonfinite;
        else if (rel > max_relres) max_relres = rel;
    }
    __device__ __forceinline__ void flush(SolvePartial* out) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int mi = __shfl_xor(max_iters, o, 64);
            max_iters = mi > max_iters ? mi : max_iters;
            n_failed += __shfl_xor(n_failed, o, 64);
            nonfinite += __shfl_xor(nonfinite, o, 64);
            const double mr = __shfl_xor(max_relres, o, 64);
            max_relres = mr > max_relres ? mr : max_relres;
        }
        if (threadIdx.x == 0) {
            SolvePartial p;
            p.max_iters = max_iters;
            p.n_failed = n_failed;
            p.nonfinite = nonfinite;
            p.pad = 0;
            p.max_relres = max_relres;
            *out = p;
        }
    }
};

}  // namespace tpfdm
