// Lane-per-block device code: one block per lane, all contractions in
// registers (used for n <= 4).
#pragma once

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

}  // namespace tpfdm
