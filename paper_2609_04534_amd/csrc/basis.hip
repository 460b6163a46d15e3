// Change of basis of a mesh plan's vectors: the fixed n x n matrix T (or
// its inverse) applied in each of the three directions of every cell
// (Sec. 3.1: the transform between the Lagrange and the Hermite-type bases,
// needed only where nodal data enter or leave).  One cell per lane, the
// cell's block in registers, three in-place pencil passes.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"

namespace tpfdm {
namespace {

template <int N>
struct BasisTab {
    double x[N * N];   // row-major: out_i = sum_j x[i][j] in_j along one axis
};

template <int N>
__global__ __launch_bounds__(64) void k_change_basis(const double* __restrict__ u, double* __restrict__ v,
                                                     int64_t nblocks, int64_t offset, int logB, BasisTab<N> X) {
    constexpr int N3 = N * N * N;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (c >= nblocks) return;
    const int64_t base = offset + block_base(c, logB, N3);
    double a[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) a[q] = u[base + (static_cast<int64_t>(q) << logB)];
    // one pass along the axis with stride st: the N values of every pencil
    auto pass = [&](int st0, int st1, int st) {
#pragma unroll
        for (int p = 0; p < N; ++p)
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const int b0 = p * st0 + r * st1;
                double t[N];
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int j = 0; j < N; ++j) s = fma(X.x[i * N + j], a[b0 + j * st], s);
                    t[i] = s;
                }
#pragma unroll
                for (int i = 0; i < N; ++i) a[b0 + i * st] = t[i];
            }
    };
    pass(N, 1, N * N);        // x (slowest): pencils over (y, z)
    pass(N * N, 1, N);        // y: pencils over (x, z)
    pass(N * N, N, 1);        // z: pencils over (x, y)
#pragma unroll
    for (int q = 0; q < N3; ++q) v[base + (static_cast<int64_t>(q) << logB)] = a[q];
}

// n >= 5: one cell per 64-thread workgroup, the block in LDS, each pass one
// output value per thread and step.
template <int N>
__global__ __launch_bounds__(64) void k_change_basis_wave(const double* __restrict__ u, double* __restrict__ v,
                                                          int64_t offset, int logB, BasisTab<N> X) {
    constexpr int N3 = N * N * N;
    __shared__ double a[N3], b[N3];
    const int64_t base = offset + block_base(blockIdx.x, logB, N3);
    for (int e = threadIdx.x; e < N3; e += 64) a[e] = u[base + (static_cast<int64_t>(e) << logB)];
    __syncthreads();
    // the three axes: out(i, j, k) = sum_m X[axis index][m] in(.. m ..)
    for (int e = threadIdx.x; e < N3; e += 64) {
        const int i = e / (N * N), jk = e % (N * N);
        double s = 0.0;
        for (int m = 0; m < N; ++m) s = fma(X.x[i * N + m], a[m * N * N + jk], s);
        b[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N3; e += 64) {
        const int i = e / (N * N), j = (e / N) % N, k = e % N;
        double s = 0.0;
        for (int m = 0; m < N; ++m) s = fma(X.x[j * N + m], b[(i * N + m) * N + k], s);
        a[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N3; e += 64) {
        const int ij = e / N, k = e % N;
        double s = 0.0;
        for (int m = 0; m < N; ++m) s = fma(X.x[k * N + m], a[ij * N + m], s);
        v[base + (static_cast<int64_t>(e) << logB)] = s;
    }
}

// The 1D factor of a change-of-basis mode: 1 (values) T, 0 (coefficients)
// T^{-1}, 2 (loads) T^T.
template <int N>
void basis_factor(const RefData& r, int mode, BasisTab<N>& X) {
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            X.x[i * N + j] = mode == 1 ? r.T[i * N + j] : mode == 0 ? r.Ti[i * N + j] : r.T[j * N + i];
}

template <int N>
tp_status change_basis_wave(const RefData& r, const GroupInfo& g, int mode, const double* u, double* v,
                            hipStream_t stream) {
    BasisTab<N> X;
    basis_factor<N>(r, mode, X);
    hipLaunchKernelGGL((k_change_basis_wave<N>), dim3(static_cast<unsigned>(g.nblocks)), dim3(64), 0, stream, u, v,
                       g.offset, g.logB, X);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TP_OK : hip_error(e, "change of basis launch");
}

}  // namespace
}  // namespace tpfdm

using namespace tpfdm;

extern "C" tp_status tp_change_basis(tp_plan* plan, int32_t to_nodal, const double* u, double* v,
                                     hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!plan->mesh) return set_error(TP_ERR_UNSUPPORTED, "change of basis needs a mesh plan");
    if (to_nodal < 0 || to_nodal > 2) return set_error(TP_ERR_ARG, "mode must be 0, 1 or 2");
    if (plan->vec_elems > 0 && (!u || !v)) return set_error(TP_ERR_ARG, "u and v must be non-null");
    if (u == v && u) return set_error(TP_ERR_ARG, "u and v must not alias");
    const GroupInfo& g = plan->groups[0];
    if (g.nblocks == 0) return TP_OK;
    if (plan->basis == TP_BASIS_LAGRANGE) {
        const hipError_t e = hipMemcpyAsync(v, u, static_cast<size_t>(plan->vec_elems) * sizeof(double),
                                            hipMemcpyDeviceToDevice, stream);
        return e == hipSuccess ? TP_OK : hip_error(e, "change of basis copy");
    }
    switch (g.n) {
        case 5: return change_basis_wave<5>(plan->ref[5], g, to_nodal, u, v, stream);
        case 6: return change_basis_wave<6>(plan->ref[6], g, to_nodal, u, v, stream);
        case 7: return change_basis_wave<7>(plan->ref[7], g, to_nodal, u, v, stream);
        case 8: return change_basis_wave<8>(plan->ref[8], g, to_nodal, u, v, stream);
        default: break;
    }
    if (g.n != 4) return set_error(TP_ERR_UNSUPPORTED, "the Hermite-type basis needs n >= 4");
    const RefData& r = plan->ref[4];
    BasisTab<4> X;
    basis_factor<4>(r, to_nodal, X);
    const unsigned grid = static_cast<unsigned>((g.nblocks + 63) / 64);
    hipLaunchKernelGGL((k_change_basis<4>), dim3(grid), dim3(64), 0, stream, u, v, g.nblocks, g.offset, g.logB, X);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TP_OK : hip_error(e, "change of basis launch");
}
