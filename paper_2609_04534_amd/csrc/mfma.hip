// Matrix-core (MFMA) kernels for n = 8 with FP16 or BF16 storage and
// operands, FP32 accumulation.
//
// At n = 8 the two inner directions of a block form a 64-wide index (j, k),
// dense enough for the 16x16x32 MFMA.  One wave processes a tile of two
// blocks as a 16-row matrix: row r = 8 w + i (block w of the tile, x-plane i)
// and column (j, k).  The lane layouts of v_mfma_f32_16x16x32 are
//   A: lane l holds A[l % 16][8 (l / 16) + v],   v = 0..7
//   B: lane l holds B[8 (l / 16) + v][l % 16]
//   D: lane l holds D[4 (l / 16) + v][l % 16],   v = 0..3
// so the A operand of row (w, i) and k-chunk c is exactly the z-pencil
// (i, j = c) of block w: 16 contiguous bytes, loaded straight from HBM.
//
// apply:  T1 = (M (x) M) u_i, T2 = (P (x) M) u_i, T3 = (M (x) P) u_i for all
//         x-planes i at once (3 x 8 MFMAs), then a = s_x T1 and
//         b = s_y T2 + s_z T3, then v = P a + M b contracts x.  D keeps 4
//         consecutive rows (x-planes) per lane; one permlane16 swap of the a
//         and b registers turns the pair into the B operand of a 16x16x32
//         MFMA with the block-diagonal A = [[P M 0 0], [0 0 P M]], so the
//         x-contraction of both blocks is one MFMA per 16 columns.
// inverse: y = (S^T (x) S^T) along (j, k) (8 MFMAs), S^T along x, scale by
//         1/(lam_a s_x + lam_b s_y + lam_c s_z), S along x (block-diagonal
//         16x16x16 MFMAs whose B layout equals the previous D layout), one
//         LDS transpose into the A layout, (S (x) S) along (j, k) (8 MFMAs).
//
// All factor operands are precomputed on the host in the per-lane register
// order of the instruction (see build_mfma_tables) and loaded once per wave.
#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "device.h"

namespace tpfdm {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Table layout (16-bit elements; one table per operator and storage type):
//   apply:   B[3][2][4][64][8]  (matrix m in {M(x)M, P(x)M, M(x)P}, K-step, N-tile, lane, v)
//            AX[64][8]          (block-diagonal x-contraction operand [P M | P M])
//   inverse: BF[2][4][64][8]    (S^T (x) S^T), BB[2][4][64][8] (S (x) S),
//            AF[64][4], AB[64][4] (block-diagonal S^T and S, 16x16x16 layout), lam[8] (float)
constexpr int kMfmaApplyHalves = 3 * 2 * 4 * 64 * 8 + 64 * 8;
constexpr int kMfmaInvHalves = 2 * 2 * 4 * 64 * 8 + 2 * 64 * 4;
constexpr int kMfmaInvBytes = kMfmaInvHalves * 2 + 8 * 4;
// Tiles of a wave whose loads are in flight ahead of the one computed
// (measured at p = 7, 32768 blocks, FP16: 2 and 4 were slower than 3).
constexpr int kPF = 3;

namespace {

// ------------------------------------------------------------ element types
template <typename TS>
struct MfmaT;
template <>
struct MfmaT<_Float16> {
    using v8 = half8_t;
    __device__ static __forceinline__ f4_t mma32(v8 a, v8 b, f4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ f4_t mma16(uint2 a, uint2 b, f4_t c) {
        half4_t ha, hb;
        __builtin_memcpy(&ha, &a, 8);
        __builtin_memcpy(&hb, &b, 8);
        return __builtin_amdgcn_mfma_f32_16x16x16f16(ha, hb, c, 0, 0, 0);
    }
    __device__ static __forceinline__ uint16_t bits(float f) {
        _Float16 h = static_cast<_Float16>(f);
        uint16_t b;
        __builtin_memcpy(&b, &h, 2);
        return b;
    }
};
template <>
struct MfmaT<bf16_t> {
    using v8 = bf8_t;
    __device__ static __forceinline__ f4_t mma32(v8 a, v8 b, f4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ f4_t mma16(uint2 a, uint2 b, f4_t c) {
        short4_t sa, sb;
        __builtin_memcpy(&sa, &a, 8);
        __builtin_memcpy(&sb, &b, 8);
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(sa, sb, c, 0, 0, 0);
    }
    __device__ static __forceinline__ uint16_t bits(float f) { return f32_to_bf16(f); }
};

template <typename TS>
__device__ __forceinline__ typename MfmaT<TS>::v8 as_v8(uint4 u) {
    typename MfmaT<TS>::v8 v;
    __builtin_memcpy(&v, &u, 16);
    return v;
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
    return static_cast<uint32_t>(lo) | (static_cast<uint32_t>(hi) << 16);
}

// Edge lengths of the block whose D rows this lane holds (block 2t + l/32),
// loaded together with the tile so that the scalings never wait on a load
// issued after the prefetches.
struct HTrip {
    double x, y, z;
};
__device__ __forceinline__ void load_tile_h(HTrip& h, const GArgs& G, int64_t t) {
    const int64_t g = 2 * t + (threadIdx.x >> 5);
    if (g < G.nblocks) {
        h.x = G.h[3 * g];
        h.y = G.h[3 * g + 1];
        h.z = G.h[3 * g + 2];
    } else {
        h.x = h.y = h.z = 1.0;
    }
}
__device__ __forceinline__ void scales_of(const HTrip& h, float& sx, float& sy, float& sz) {
    sx = static_cast<float>(h.y * h.z / h.x);
    sy = static_cast<float>(h.x * h.z / h.y);
    sz = static_cast<float>(h.x * h.y / h.z);
}

// Unconditional versions for tiles whose two blocks both exist: every
// iteration of the main loop then issues the same memory instructions, which
// lets the compiler wait only for the oldest prefetched tile.
__device__ __forceinline__ void load_full_h(HTrip& h, const GArgs& G, int64_t t) {
    const int64_t g = 2 * t + (threadIdx.x >> 5);
    h.x = G.h[3 * g];
    h.y = G.h[3 * g + 1];
    h.z = G.h[3 * g + 2];
}
template <typename TS>
__device__ __forceinline__ void load_full_a(uint4 (&a)[2], const TS* __restrict__ u, const GArgs& G, int64_t t) {
    const int l = threadIdx.x;
    const int row = l & 15;
    const uint4* p = reinterpret_cast<const uint4*>(u + G.offset + (2 * t + (row >> 3)) * 512 + (row & 7) * 64);
    a[0] = p[(l >> 4)];
    a[1] = p[4 + (l >> 4)];
}

// A operands of one tile: the z-pencils of row (w, i) = (l%16 / 8, l%16 % 8)
// for k-chunks j = 4 s + l / 16 (s = 0, 1).  Missing blocks read as zero.
template <typename TS>
__device__ __forceinline__ void load_tile_a(uint4 (&a)[2], const TS* __restrict__ u, const GArgs& G, int64_t t) {
    const int l = threadIdx.x;
    const int row = l & 15;
    const int64_t g = 2 * t + (row >> 3);
    const int i = row & 7;
    if (g < G.nblocks) {
        const uint4* p = reinterpret_cast<const uint4*>(u + G.offset + g * 512 + i * 64);
        a[0] = p[(l >> 4)];
        a[1] = p[4 + (l >> 4)];
    } else {
        a[0] = make_uint4(0, 0, 0, 0);
        a[1] = make_uint4(0, 0, 0, 0);
    }
}

// Output staging: the D tiles of one tile (16 rows x 64 columns) are written
// to LDS in D layout and read back in A layout (16 contiguous bytes per lane:
// row l % 16, columns 8 (l / 16) + 32 s), so every lane stores two 16-byte
// chunks of one x-plane row.
struct OutTile {
    uint16_t v[16][72];
};

__device__ __forceinline__ void out_put(OutTile& o, int nt, uint16_t b0, uint16_t b1, uint16_t b2, uint16_t b3) {
    const int l = threadIdx.x;
    const int col = 16 * nt + (l & 15);
    const int r = 4 * (l >> 4);
    o.v[r][col] = b0;
    o.v[r + 1][col] = b1;
    o.v[r + 2][col] = b2;
    o.v[r + 3][col] = b3;
}

template <bool FULL, typename TS>
__device__ __forceinline__ void out_flush(OutTile& o, TS* __restrict__ v, const GArgs& G, int64_t t) {
    wave_sync();
    const int l = threadIdx.x;
    const int row = l & 15;
    const int64_t g = 2 * t + (row >> 3);
    uint4 c0, c1;
    __builtin_memcpy(&c0, &o.v[row][8 * (l >> 4)], 16);
    __builtin_memcpy(&c1, &o.v[row][8 * (l >> 4) + 32], 16);
    wave_sync();
    if (FULL || g < G.nblocks) {
        uint4* p = reinterpret_cast<uint4*>(v + G.offset + g * 512 + (row & 7) * 64);
        p[l >> 4] = c0;
        p[4 + (l >> 4)] = c1;
    }
}

template <typename TS>
__global__ __launch_bounds__(64, 2) void k_apply_mfma(const TS* __restrict__ u, TS* __restrict__ v, GArgs G,
                                                      const uint16_t* __restrict__ tab, int64_t ntiles) {
    using T = MfmaT<TS>;
    const int l = threadIdx.x;
    // factor operands: 24 B registers (3 matrices x 2 K-steps x 4 N-tiles) and AX
    uint4 B[3][2][4];
    const uint4* tb = reinterpret_cast<const uint4*>(tab);
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) B[m][s][nt] = tb[((m * 2 + s) * 4 + nt) * 64 + l];
    const uint4 AX = tb[3 * 2 * 4 * 64 + l];
    __shared__ OutTile ot;
    // tile body: cur = A operands, sx, sy, sz = scalings of the lane's block
    auto tile = [&](const uint4 (&cur)[2], float sx, float sy, float sz, int64_t t) {
        // per-lane block of the D rows: block 2t + l/32
        const typename T::v8 a0 = as_v8<TS>(cur[0]), a1 = as_v8<TS>(cur[1]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f4_t z = {0.f, 0.f, 0.f, 0.f};
            f4_t t1 = T::mma32(a0, as_v8<TS>(B[0][0][nt]), z);
            t1 = T::mma32(a1, as_v8<TS>(B[0][1][nt]), t1);
            f4_t t2 = T::mma32(a0, as_v8<TS>(B[1][0][nt]), z);
            t2 = T::mma32(a1, as_v8<TS>(B[1][1][nt]), t2);
            f4_t t3 = T::mma32(a0, as_v8<TS>(B[2][0][nt]), z);
            t3 = T::mma32(a1, as_v8<TS>(B[2][1][nt]), t3);
            // a = s_x T1, b = s_y T2 + s_z T3, then swap rows 1,3 of a with
            // rows 0,2 of b: lanes of row group g then hold k-group g of the
            // block-diagonal x-contraction ([a0; b0; a1; b1], 8 planes each)
            uint32_t lo[4], hi[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float av = sx * t1[q];
                const float bv = fmaf(sy, t2[q], sz * t3[q]);
                const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(av), __float_as_uint(bv), false,
                                                                 false);
                lo[q] = sw[0];
                hi[q] = sw[1];
            }
            uint4 bx;
            bx.x = pack2(T::bits(__uint_as_float(lo[0])), T::bits(__uint_as_float(lo[1])));
            bx.y = pack2(T::bits(__uint_as_float(lo[2])), T::bits(__uint_as_float(lo[3])));
            bx.z = pack2(T::bits(__uint_as_float(hi[0])), T::bits(__uint_as_float(hi[1])));
            bx.w = pack2(T::bits(__uint_as_float(hi[2])), T::bits(__uint_as_float(hi[3])));
            const f4_t vout = T::mma32(as_v8<TS>(AX), as_v8<TS>(bx), z);
            out_put(ot, nt, T::bits(vout[0]), T::bits(vout[1]), T::bits(vout[2]), T::bits(vout[3]));
        }
    };
    const int64_t G2 = gridDim.x;
    const int64_t nfull = G.nblocks / 2;  // tiles with both blocks present
    int64_t t = blockIdx.x;
    if (t < nfull) {
        const int64_t tlast = t + ((nfull - 1 - t) / G2) * G2;  // this wave's last full tile
        uint4 ring[kPF][2];
        HTrip hring[kPF];
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            const int64_t tp = std::min(t + p * G2, tlast);
            load_full_h(hring[p], G, tp);
            load_full_a(ring[p], u, G, tp);
        }
        // the ring slot is a compile-time index (the main loop is unrolled
        // kPF times and has no early exit, so every pass issues the same
        // memory instructions and each wait covers only the oldest tile's
        // loads, not the prefetches and stores behind it); prefetches past
        // the wave's last tile re-read that tile
        const int64_t cnt = (tlast - t) / G2 + 1;   // tiles of this wave
        int64_t i = 0;
        for (; i + kPF <= cnt; i += kPF) {
#pragma unroll
            for (int slot = 0; slot < kPF; ++slot) {
                // the slot is refilled only after its tile has consumed it,
                // so the new loads land in the slot's own registers (a copy
                // out of registers with a load in flight would wait for it);
                // no instruction crosses into the next slot's tile, which
                // would wait for that younger tile's loads
                __builtin_amdgcn_sched_barrier(0);
                float sx, sy, sz;
                scales_of(hring[slot], sx, sy, sz);
                const int64_t tn = std::min(t + kPF * G2, tlast);
                load_full_h(hring[slot], G, tn);
                tile(ring[slot], sx, sy, sz, t);
                load_full_a(ring[slot], u, G, tn);
                out_flush<true>(ot, v, G, t);
                t += G2;
            }
        }
        // the last cnt - i < kPF tiles are already in ring slots 0, 1, ...
#pragma unroll
        for (int slot = 0; slot < kPF - 1; ++slot) {
            if (i + slot < cnt) {
                float sx, sy, sz;
                scales_of(hring[slot], sx, sy, sz);
                tile(ring[slot], sx, sy, sz, t);
                out_flush<true>(ot, v, G, t);
                t += G2;
            }
        }
    }
    // the tile holding the last block of an odd count
    if ((G.nblocks & 1) && static_cast<int64_t>(blockIdx.x) == nfull % G2) {
        uint4 cur[2];
        HTrip h;
        load_tile_h(h, G, nfull);
        load_tile_a(cur, u, G, nfull);
        float sx, sy, sz;
        scales_of(h, sx, sy, sz);
        tile(cur, sx, sy, sz, nfull);
        out_flush<false>(ot, v, G, nfull);
    }
}

template <typename TS>
__global__ __launch_bounds__(64, 2) void k_inverse_mfma(const TS* __restrict__ r, TS* __restrict__ x, GArgs G,
                                                        const uint16_t* __restrict__ tab, int64_t ntiles) {
    using T = MfmaT<TS>;
    __shared__ uint16_t tr[16][72];  // transpose tile: 16 rows x 64 columns (+8 pad)
    __shared__ float slam[8];
    const int l = threadIdx.x;
    const uint4* tb = reinterpret_cast<const uint4*>(tab);
    uint4 BF[2][4], BB[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            BF[s][nt] = tb[(s * 4 + nt) * 64 + l];
            BB[s][nt] = tb[(8 + s * 4 + nt) * 64 + l];
        }
    const uint2* t2p = reinterpret_cast<const uint2*>(tab + 2 * 2 * 4 * 64 * 8);
    const uint2 AF = t2p[l], AB = t2p[64 + l];
    const float* lamp = reinterpret_cast<const float*>(tab + kMfmaInvHalves);
    if (l < 8) slam[l] = lamp[l];
    wave_sync();
    // spectral indices of this lane's D entries: rows a = 4 (l/16 % 2) + q, column (b, c)
    const int a0 = 4 * ((l >> 4) & 1);
    float la[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) la[q] = slam[a0 + q];
    __shared__ OutTile ot;
    // tile body: cur = A operands, sx, sy, sz = scalings of the lane's block
    auto tile = [&](const uint4 (&cur)[2], float sx, float sy, float sz, int64_t t) {
        const typename T::v8 a0v = as_v8<TS>(cur[0]), a1v = as_v8<TS>(cur[1]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f4_t z = {0.f, 0.f, 0.f, 0.f};
            // (S^T (x) S^T) along (j, k)
            f4_t y = T::mma32(a0v, as_v8<TS>(BF[0][nt]), z);
            y = T::mma32(a1v, as_v8<TS>(BF[1][nt]), y);
            // S^T along x (block-diagonal 16x16x16; B layout = D layout)
            uint2 bq;
            bq.x = pack2(T::bits(y[0]), T::bits(y[1]));
            bq.y = pack2(T::bits(y[2]), T::bits(y[3]));
            f4_t w = T::mma16(AF, bq, z);
            // diagonal scaling: column (b, c) = 16 nt + l%16
            const int col = 16 * nt + (l & 15);
            const float mu_bc = slam[col >> 3] * sy + slam[col & 7] * sz;
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] *= recip(fmaf(la[q], sx, mu_bc));
            // S along x
            bq.x = pack2(T::bits(w[0]), T::bits(w[1]));
            bq.y = pack2(T::bits(w[2]), T::bits(w[3]));
            const f4_t zz = T::mma16(AB, bq, z);
            // into the transpose tile: row 4 (l/16) + q, column col
#pragma unroll
            for (int q = 0; q < 4; ++q) tr[4 * (l >> 4) + q][col] = T::bits(zz[q]);
        }
        wave_sync();
        // A layout: row l%16, columns 8 (l/16) + 32 s .. + 7
        uint4 za[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const uint16_t* rowp = &tr[l & 15][8 * (l >> 4) + 32 * s];
            uint4 val;
            __builtin_memcpy(&val, rowp, 16);
            za[s] = val;
        }
        wave_sync();
        const typename T::v8 z0 = as_v8<TS>(za[0]), z1 = as_v8<TS>(za[1]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f4_t z = {0.f, 0.f, 0.f, 0.f};
            f4_t o = T::mma32(z0, as_v8<TS>(BB[0][nt]), z);
            o = T::mma32(z1, as_v8<TS>(BB[1][nt]), o);
            out_put(ot, nt, T::bits(o[0]), T::bits(o[1]), T::bits(o[2]), T::bits(o[3]));
        }
    };
    const int64_t G2 = gridDim.x;
    const int64_t nfull = G.nblocks / 2;  // tiles with both blocks present
    int64_t t = blockIdx.x;
    if (t < nfull) {
        const int64_t tlast = t + ((nfull - 1 - t) / G2) * G2;  // this wave's last full tile
        uint4 ring[kPF][2];
        HTrip hring[kPF];
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            const int64_t tp = std::min(t + p * G2, tlast);
            load_full_h(hring[p], G, tp);
            load_full_a(ring[p], r, G, tp);
        }
        // the ring slot is a compile-time index (the main loop is unrolled
        // kPF times and has no early exit, so every pass issues the same
        // memory instructions and each wait covers only the oldest tile's
        // loads, not the prefetches and stores behind it); prefetches past
        // the wave's last tile re-read that tile
        const int64_t cnt = (tlast - t) / G2 + 1;   // tiles of this wave
        int64_t i = 0;
        for (; i + kPF <= cnt; i += kPF) {
#pragma unroll
            for (int slot = 0; slot < kPF; ++slot) {
                // the slot is refilled only after its tile has consumed it,
                // so the new loads land in the slot's own registers (a copy
                // out of registers with a load in flight would wait for it);
                // no instruction crosses into the next slot's tile, which
                // would wait for that younger tile's loads
                __builtin_amdgcn_sched_barrier(0);
                float sx, sy, sz;
                scales_of(hring[slot], sx, sy, sz);
                const int64_t tn = std::min(t + kPF * G2, tlast);
                load_full_h(hring[slot], G, tn);
                tile(ring[slot], sx, sy, sz, t);
                load_full_a(ring[slot], r, G, tn);
                out_flush<true>(ot, x, G, t);
                t += G2;
            }
        }
        // the last cnt - i < kPF tiles are already in ring slots 0, 1, ...
#pragma unroll
        for (int slot = 0; slot < kPF - 1; ++slot) {
            if (i + slot < cnt) {
                float sx, sy, sz;
                scales_of(hring[slot], sx, sy, sz);
                tile(ring[slot], sx, sy, sz, t);
                out_flush<true>(ot, x, G, t);
                t += G2;
            }
        }
    }
    // the tile holding the last block of an odd count
    if ((G.nblocks & 1) && static_cast<int64_t>(blockIdx.x) == nfull % G2) {
        uint4 cur[2];
        HTrip h;
        load_tile_h(h, G, nfull);
        load_tile_a(cur, r, G, nfull);
        float sx, sy, sz;
        scales_of(h, sx, sy, sz);
        tile(cur, sx, sy, sz, nfull);
        out_flush<false>(ot, x, G, nfull);
    }
}

tp_status check_m(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

int64_t mgrid(const Plan& plan, const void* kern) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, 0) != hipSuccess || occ <= 0) occ = 8;
    return static_cast<int64_t>(plan.cus) * occ;
}

// ------------------------------------------------------------ host tables
uint16_t host_f16(double d) {
    _Float16 h = static_cast<_Float16>(static_cast<float>(d));
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}
uint16_t host_bf16(double d) {
    float f = static_cast<float>(d);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

}  // namespace

// Per-lane operand tables for the n = 8 MFMA kernels.
//  apply (P = K or A_hat): yz matrices Mat_m[(j,k)][(j',k')], B[k = (j',k')][n = (j,k)] = Mat_m[n][k].
//  inverse: B_fwd[k = (j,k)][n = (b,c)] = S[j][b] S[k][c]; B_bwd[k = (b,c)][n = (j,k)] = S[j][b] S[k][c].
bool build_mfma_tables(const double* M, const double* P, const double* S, const double* lam, bool bf16,
                       std::vector<uint16_t>* apply, std::vector<uint8_t>* inverse) {
    const int n = 8;
    auto cvt = [&](double d) { return bf16 ? host_bf16(d) : host_f16(d); };
    if (apply) {
        apply->assign(kMfmaApplyHalves, 0);
        for (int m = 0; m < 3; ++m) {
            const double* Ay = (m == 1) ? P : M;   // factor on y
            const double* Az = (m == 2) ? P : M;   // factor on z
            for (int s = 0; s < 2; ++s)
                for (int nt = 0; nt < 4; ++nt)
                    for (int l = 0; l < 64; ++l)
                        for (int v = 0; v < 8; ++v) {
                            const int kk = 32 * s + 8 * (l / 16) + v;   // (j', k')
                            const int nn = 16 * nt + (l % 16);          // (j, k)
                            const int j = nn / n, k = nn % n, jp = kk / n, kp = kk % n;
                            (*apply)[(((m * 2 + s) * 4 + nt) * 64 + l) * 8 + v] =
                                cvt(Ay[j * n + jp] * Az[k * n + kp]);
                        }
        }
        // AX: block-diagonal [[P M 0 0], [0 0 P M]], 16 x 32, lane l: row l%16, k = 8 (l/16) + v
        for (int l = 0; l < 64; ++l)
            for (int v = 0; v < 8; ++v) {
                const int row = l % 16, g = l / 16;
                const int blk = row / 8, i = row % 8;
                double val = 0.0;
                if (g / 2 == blk) val = (g % 2 == 0) ? P[i * n + v] : M[i * n + v];
                (*apply)[3 * 2 * 4 * 64 * 8 + l * 8 + v] = cvt(val);
            }
    }
    if (inverse) {
        std::vector<uint16_t> h(kMfmaInvHalves, 0);
        for (int d = 0; d < 2; ++d)
            for (int s = 0; s < 2; ++s)
                for (int nt = 0; nt < 4; ++nt)
                    for (int l = 0; l < 64; ++l)
                        for (int v = 0; v < 8; ++v) {
                            const int kk = 32 * s + 8 * (l / 16) + v;
                            const int nn = 16 * nt + (l % 16);
                            // forward: k = (j,k) data index, n = (b,c) spectral; backward: the reverse
                            const int jk = d == 0 ? kk : nn, bc = d == 0 ? nn : kk;
                            const int j = jk / n, k = jk % n, b = bc / n, c = bc % n;
                            h[(((d * 2 + s) * 4 + nt) * 64 + l) * 8 + v] = cvt(S[j * n + b] * S[k * n + c]);
                        }
        // AF, AB: block-diagonal S^T and S in the 16x16x16 layout (lane l: row l%16, k = 4 (l/16) + v)
        for (int d = 0; d < 2; ++d)
            for (int l = 0; l < 64; ++l)
                for (int v = 0; v < 4; ++v) {
                    const int row = l % 16, k = 4 * (l / 16) + v;
                    double val = 0.0;
                    if (row / 8 == k / 8) {
                        const int rr = row % 8, kk2 = k % 8;
                        val = d == 0 ? S[kk2 * n + rr] : S[rr * n + kk2];  // S^T[a][i] = S[i][a]
                    }
                    h[2 * 2 * 4 * 64 * 8 + d * 256 + l * 4 + v] = cvt(val);
                }
        inverse->assign(kMfmaInvBytes, 0);
        std::memcpy(inverse->data(), h.data(), h.size() * 2);
        float lf[8];
        for (int i = 0; i < 8; ++i) lf[i] = static_cast<float>(lam[i]);
        std::memcpy(inverse->data() + h.size() * 2, lf, sizeof(lf));
    }
    return true;
}

bool mfma_eligible(const GroupInfo& g, tp_dtype dt, const void* a, const void* b) {
    if (g.n != 8 || g.logB != 0 || (dt != TP_F16 && dt != TP_BF16)) return false;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a) + static_cast<uintptr_t>(g.offset) * 2;
    const uintptr_t pb = reinterpret_cast<uintptr_t>(b) + static_cast<uintptr_t>(g.offset) * 2;
    return pa % 16 == 0 && pb % 16 == 0;
}

tp_status launch_apply_mfma(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v, tp_dtype dt,
                            hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    const int et = dt == TP_BF16 ? 1 : 0;
    const uint16_t* tab = static_cast<const uint16_t*>(plan.mfma_apply_dev[op == TP_OP_CELL ? 1 : 0][et]);
    if (!tab) return set_error(TP_ERR_STATE, "MFMA tables missing");
    const int64_t ntiles = (g.nblocks + 1) / 2;
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    if (dt == TP_F16) {
        static int64_t gc = 0;
        if (gc == 0) gc = mgrid(plan, reinterpret_cast<const void*>(&k_apply_mfma<_Float16>));
        hipLaunchKernelGGL((k_apply_mfma<_Float16>), dim3(static_cast<unsigned>(std::min(gc, ntiles))), dim3(64), 0,
                           s, static_cast<const _Float16*>(u), static_cast<_Float16*>(v), a, tab, ntiles);
    } else {
        static int64_t gc = 0;
        if (gc == 0) gc = mgrid(plan, reinterpret_cast<const void*>(&k_apply_mfma<bf16_t>));
        hipLaunchKernelGGL((k_apply_mfma<bf16_t>), dim3(static_cast<unsigned>(std::min(gc, ntiles))), dim3(64), 0, s,
                           static_cast<const bf16_t*>(u), static_cast<bf16_t*>(v), a, tab, ntiles);
    }
    return check_m("apply (MFMA) launch");
}

tp_status launch_inverse_mfma(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                              hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    const int et = dt == TP_BF16 ? 1 : 0;
    const uint16_t* tab = static_cast<const uint16_t*>(plan.mfma_inv_dev[et]);
    if (!tab) return set_error(TP_ERR_STATE, "MFMA tables missing");
    const int64_t ntiles = (g.nblocks + 1) / 2;
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    if (dt == TP_F16) {
        static int64_t gc = 0;
        if (gc == 0) gc = mgrid(plan, reinterpret_cast<const void*>(&k_inverse_mfma<_Float16>));
        hipLaunchKernelGGL((k_inverse_mfma<_Float16>), dim3(static_cast<unsigned>(std::min(gc, ntiles))), dim3(64),
                           0, s, static_cast<const _Float16*>(r), static_cast<_Float16*>(x), a, tab, ntiles);
    } else {
        static int64_t gc = 0;
        if (gc == 0) gc = mgrid(plan, reinterpret_cast<const void*>(&k_inverse_mfma<bf16_t>));
        hipLaunchKernelGGL((k_inverse_mfma<bf16_t>), dim3(static_cast<unsigned>(std::min(gc, ntiles))), dim3(64), 0,
                           s, static_cast<const bf16_t*>(r), static_cast<bf16_t*>(x), a, tab, ntiles);
    }
    return check_m("apply_inverse (MFMA) launch");
}

}  // namespace tpfdm
