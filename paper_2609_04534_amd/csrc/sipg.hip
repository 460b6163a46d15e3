// Launch of the coupled SIPG operator of a mesh plan (device code in sipg.h).
#include "sipg.h"

namespace tpfdm {

namespace {

// One cell per lane (n <= 4).  The cell's own block is read with cached
// loads (it is also a face source of its neighbours); v is streamed out.
template <int N, typename TS, typename TC, bool NT, int LB, bool HERM = false>
__global__ __launch_bounds__(64, 2) void k_sipg_lane(const TS* __restrict__ u, TS* __restrict__ v, MeshArgs G,
                                                   Pair<N, TC> R, FaceRef<N, TC> F) {
    constexpr int N3 = N * N * N;
    __shared__ TC sa[N * N][64], sbt[N * N][64];
    const int64_t c = static_cast<int64_t>(lane_tile(blockIdx.x, gridDim.x, plane_tiles<N, TS, HERM>(G))) * 64 + threadIdx.x;
    if (c >= G.ncells) return;
    TC acc[N3];
    sipg_cell<N, TS, TC, LB, HERM>(u, G, R, F, c, acc, sa, sbt);
    const int lb = LB >= 0 ? LB : G.logB;
    TS* vb = v + G.offset + block_base(c, lb, N3);
#pragma unroll
    for (int q = 0; q < N3; ++q) stv<NT>(vb + (static_cast<int64_t>(q) << lb), acc[q]);
}

// One cell per wave (n >= 5); HERM: the Hermite-type basis.
template <int N, typename T, bool VP, bool HERM>
__global__ __launch_bounds__(64, 2) void k_sipg_wave(const T* __restrict__ u, T* __restrict__ v, MeshArgs G,
                                                  const T* __restrict__ tab, FaceRef<N, T> F) {
    constexpr int TAB = 2 * (EOShape<N>::SE + EOShape<N>::SO);
    __shared__ WaveLds<N, T> L;
    // FP64: the tables are read at wave-uniform global addresses (scalar
    // loads; in VGPRs they would take half the register file, from LDS they
    // would compete with the slab traffic); FP32: from registers
    T TB[sizeof(T) == 8 ? 1 : TAB];
    const T* tb = TB;
    if constexpr (sizeof(T) == 8) {
        tb = tab;
    } else {
        load_table<T, TAB>(TB, tab, nullptr);   // FP32: straight from the global table
    }
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x);
    T y[N];
    wave_sipg_cell<N, T, VP, HERM>(u, G, tb, F, c, L, y);
    const Pencil<N> pc(1);
    if (pc.act) {
        T* vb = v + G.offset + block_base(c, G.logB, N * N * N);
        constexpr bool kWholeLines = (N * N * sizeof(T)) % 128 == 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T* o = vb + (static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << G.logB);
            if constexpr (kWholeLines) stg(o, y[i]);
            else stc(o, y[i]);
        }
    }
}

tp_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}
template <int N, typename TS, typename TC>
tp_status sipg_lane_n(const Plan& plan, const MeshArgs& G, bool face_only, const void* u, void* v, hipStream_t s) {
    Pair<N, TC> R;
    FaceRef<N, TC> F;
    sipg_tables<N, TC>(plan, face_only, R, F);
    const unsigned grid = static_cast<unsigned>((G.ncells + 63) / 64);
    const TS* ui = static_cast<const TS*>(u);
    TS* vo = static_cast<TS*>(v);
    if constexpr (N == 4) {   // the Hermite-type basis: two-layer face terms
        if (plan.basis == TP_BASIS_HERMITE) {
            if (G.logB == 6)
                hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, true, 6, true>), dim3(grid), dim3(64), 0, s, ui, vo, G, R,
                                   F);
            else if (lane_whole_lines<TS>(G.logB))
                hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, true, -1, true>), dim3(grid), dim3(64), 0, s, ui, vo, G,
                                   R, F);
            else
                hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, false, -1, true>), dim3(grid), dim3(64), 0, s, ui, vo, G,
                                   R, F);
            return check_launch("SIPG apply launch");
        }
    }
    if (G.logB == 6)
        hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, true, 6>), dim3(grid), dim3(64), 0, s, ui, vo, G, R, F);
    else if (lane_whole_lines<TS>(G.logB))
        hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, true, -1>), dim3(grid), dim3(64), 0, s, ui, vo, G, R, F);
    else
        hipLaunchKernelGGL((k_sipg_lane<N, TS, TC, false, -1>), dim3(grid), dim3(64), 0, s, ui, vo, G, R, F);
    return check_launch("SIPG apply launch");
}

template <int N, typename T>
tp_status sipg_wave_n(const Plan& plan, const MeshArgs& G, bool face_only, const void* u, void* v, hipStream_t s) {
    Pair<N, T> R;
    FaceRef<N, T> F;
    sipg_tables<N, T>(plan, face_only, R, F);
    const T* tab = reinterpret_cast<const T*>(eo_table(plan, N, face_only ? EO_APPLY_F : EO_APPLY_A,
                                                       sizeof(T) == 8 ? 0 : 1));
    const unsigned grid = static_cast<unsigned>(G.ncells);
    const T* ui = static_cast<const T*>(u);
    T* vo = static_cast<T*>(v);
    // 16-byte pencils: block-contiguous layout and an aligned vector
    const bool vp = G.logB == 0 && (reinterpret_cast<uintptr_t>(ui + G.offset) % 16 == 0) &&
                    (N * sizeof(T)) % 16 == 0;
    if (plan.basis == TP_BASIS_HERMITE) {
        flip_face_ref<N, T>(F);
        if (vp)
            hipLaunchKernelGGL((k_sipg_wave<N, T, true, true>), dim3(grid), dim3(64), 0, s, ui, vo, G, tab, F);
        else
            hipLaunchKernelGGL((k_sipg_wave<N, T, false, true>), dim3(grid), dim3(64), 0, s, ui, vo, G, tab, F);
    } else if (vp) {
        hipLaunchKernelGGL((k_sipg_wave<N, T, true, false>), dim3(grid), dim3(64), 0, s, ui, vo, G, tab, F);
    } else {
        hipLaunchKernelGGL((k_sipg_wave<N, T, false, false>), dim3(grid), dim3(64), 0, s, ui, vo, G, tab, F);
    }
    return check_launch("SIPG apply launch");
}

template <typename TS, typename TC>
tp_status sipg_dispatch(const Plan& plan, const MeshArgs& G, int n, bool face_only, const void* u, void* v,
                        hipStream_t s) {
    switch (n) {
        case 2: return sipg_lane_n<2, TS, TC>(plan, G, face_only, u, v, s);
        case 3: return sipg_lane_n<3, TS, TC>(plan, G, face_only, u, v, s);
        case 4: return sipg_lane_n<4, TS, TC>(plan, G, face_only, u, v, s);
        case 5: return sipg_wave_n<5, TC>(plan, G, face_only, u, v, s);
        case 6: return sipg_wave_n<6, TC>(plan, G, face_only, u, v, s);
        case 7: return sipg_wave_n<7, TC>(plan, G, face_only, u, v, s);
        case 8: return sipg_wave_n<8, TC>(plan, G, face_only, u, v, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

}  // namespace

tp_status launch_sipg(const Plan& plan, const GroupInfo& g, bool face_only, const void* u, void* v, tp_dtype dt,
                      hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    const MeshArgs G = mesh_args(plan, g);
    switch (dt) {
        case TP_F64: return sipg_dispatch<double, double>(plan, G, g.n, face_only, u, v, s);
        case TP_F32: return sipg_dispatch<float, float>(plan, G, g.n, face_only, u, v, s);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "the SIPG operator supports TP_F64 and TP_F32");
}

}  // namespace tpfdm
