// C-ABI entry points of libtpfdm: argument checking, plan ownership and
// dispatch to the kernel launchers.  See include/tpfdm.h for the contract.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace tpfdm {

namespace {
thread_local std::string g_last_error;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}
int esize_of(tp_dtype dt) {
    switch (dt) {
        case TP_F64: return 8;
        case TP_F32: return 4;
        case TP_F16: return 2;
        case TP_BF16: return 2;
    }
    return 0;
}
bool use_lane(const Plan& p, const GroupInfo& g) {
    return !g.factors && g.n <= kLaneMaxN && p.mapping != TP_MAP_WAVE;
}
bool use_mfma(const Plan& p, const GroupInfo& g, tp_dtype dt, const void* a, const void* b) {
    return p.mapping != TP_MAP_WAVE && mfma_eligible(g, dt, a, b);
}
// Kernel family of a group's apply / apply_inverse / solve: the autotuned
// choice when it applies to this call, else the default rule.
int apply_kind(const Plan& p, const GroupInfo& g, tp_dtype dt, const void* a, const void* b) {
    if (g.factors) return KIND_GENERAL;
    const int t = g.tune_apply[dt];
    if (t == KIND_LANE && g.n <= kLaneMaxN) return KIND_LANE;
    if (t == KIND_MFMA && mfma_eligible(g, dt, a, b)) return KIND_MFMA;
    if (t == KIND_WAVE) return KIND_WAVE;
    return use_lane(p, g) ? KIND_LANE : use_mfma(p, g, dt, a, b) ? KIND_MFMA : KIND_WAVE;
}
int inverse_kind(const Plan& p, const GroupInfo& g, tp_dtype dt, const void* a, const void* b) {
    if (p.factor_mode == TP_FACTOR_GENERAL) return KIND_GENERAL;
    const int t = g.tune_inverse[dt];
    if (t == KIND_LANE && g.n <= kLaneMaxN) return KIND_LANE;
    if (t == KIND_MFMA && mfma_eligible(g, dt, a, b)) return KIND_MFMA;
    if (t == KIND_WAVE) return KIND_WAVE;
    return use_lane(p, g) ? KIND_LANE : use_mfma(p, g, dt, a, b) ? KIND_MFMA : KIND_WAVE;
}
int solve_kind(const Plan& p, const GroupInfo& g) {
    if (p.factor_mode == TP_FACTOR_GENERAL) return KIND_GENERAL;
    if (g.tune_solve == KIND_LANE && g.n <= kLaneMaxN && !g.factors) return KIND_LANE;
    if (g.tune_solve == KIND_WAVE) return KIND_WAVE;
    return g.lane_solve ? KIND_LANE : KIND_WAVE;
}

bool valid_dtype(int dt) { return dt >= TP_F64 && dt <= TP_BF16; }
bool valid_op(int op) { return op == TP_OP_NEUMANN || op == TP_OP_CELL; }
bool coupled_op(int op) { return op == TP_OP_SIPG || op == TP_OP_SIPG_FACE; }

}  // namespace

tp_status set_error(tp_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

tp_status hip_error(int err, const char* what) {
    const char* s = hipGetErrorString(static_cast<hipError_t>(err));
    return set_error(TP_ERR_HIP, std::string(what) + ": " + (s ? s : "unknown HIP error"));
}

// Frees the per-block eigen-decompositions (and with all, the factors).
static void free_block_factors(GroupInfo& g, bool all) {
    if (g.eig) (void)hipFree(g.eig), g.eig = nullptr;
    if (g.eig32) (void)hipFree(g.eig32), g.eig32 = nullptr;
    if (all || !g.factors) {
        if (g.fac) (void)hipFree(g.fac), g.fac = nullptr;
        if (g.fac32) (void)hipFree(g.fac32), g.fac32 = nullptr;
    }
}

static void free_plan_memory(Plan* p) {
    for (auto& g : p->groups) {
        if (g.h) (void)hipFree(g.h), g.h = nullptr;
        free_block_factors(g, true);
    }
    if (p->summary_dev) (void)hipFree(p->summary_dev), p->summary_dev = nullptr;
    if (p->summary_host) (void)hipHostFree(p->summary_host), p->summary_host = nullptr;
    p->summary_host_dev = nullptr;
    if (p->partials_dev) (void)hipFree(p->partials_dev), p->partials_dev = nullptr;
    if (p->segs_dev) (void)hipFree(p->segs_dev), p->segs_dev = nullptr;
    if (p->eo_dev) (void)hipFree(p->eo_dev), p->eo_dev = nullptr;
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j)
            if (p->mfma_apply_dev[i][j]) (void)hipFree(p->mfma_apply_dev[i][j]), p->mfma_apply_dev[i][j] = nullptr;
        if (p->mfma_inv_dev[i]) (void)hipFree(p->mfma_inv_dev[i]), p->mfma_inv_dev[i] = nullptr;
    }
}

static tp_status alloc_dev(void** ptr, size_t bytes, const char* what) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return set_error(TP_ERR_OOM, std::string("out of device memory: ") + what);
    }
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

// Uploads a host FP64 array to new device memory as FP64 and as FP32.
static tp_status upload_both(const std::vector<double>& h, double** d64, float** d32, const char* what) {
    tp_status st = alloc_dev(reinterpret_cast<void**>(d64), h.size() * sizeof(double), what);
    if (st != TP_OK) return st;
    hipError_t e = hipMemcpy(*d64, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, what);
    std::vector<float> f(h.begin(), h.end());
    st = alloc_dev(reinterpret_cast<void**>(d32), f.size() * sizeof(float), what);
    if (st != TP_OK) return st;
    e = hipMemcpy(*d32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

// Copies a factor group's M and P (host or device, [nblocks][3][n][n]) into
// plan-owned memory interleaved as [nblocks][3][2][n][n].
static tp_status copy_factors(GroupInfo& g, const double* M, const double* P, int gi) {
    const size_t nn = static_cast<size_t>(g.n) * g.n;
    const size_t cnt = static_cast<size_t>(g.nblocks) * 3 * nn;
    std::vector<double> hm(cnt), hp(cnt);
    hipError_t e = hipMemcpy(hm.data(), M, cnt * sizeof(double), hipMemcpyDefault);
    if (e == hipSuccess) e = hipMemcpy(hp.data(), P, cnt * sizeof(double), hipMemcpyDefault);
    if (e != hipSuccess) return hip_error(e, "copy of block factors");
    std::vector<double> fac(2 * cnt);
    for (size_t bd = 0; bd < static_cast<size_t>(g.nblocks) * 3; ++bd)
        for (size_t e2 = 0; e2 < nn; ++e2) {
            const double m = hm[bd * nn + e2], q = hp[bd * nn + e2];
            if (!std::isfinite(m) || !std::isfinite(q))
                return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": non-finite factor in block " +
                                                 std::to_string(bd / 3));
            fac[(2 * bd) * nn + e2] = m;
            fac[(2 * bd + 1) * nn + e2] = q;
        }
    return upload_both(fac, &g.fac, &g.fac32, "block factors");
}

tp_status upload_eo(Plan& plan, int n, int tab, const double* vals, int count) {
    if (count > kEOSlot) return set_error(TP_ERR_UNSUPPORTED, "even-odd table too large");
    float f[kEOSlot];
    for (int i = 0; i < count; ++i) f[i] = static_cast<float>(vals[i]);
    hipError_t e = hipMemcpy(const_cast<void*>(eo_table(plan, n, tab, 0)), vals, count * sizeof(double),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(const_cast<void*>(eo_table(plan, n, tab, 1)), f, count * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "upload of even-odd tables");
    return TP_OK;
}

}  // namespace tpfdm

using namespace tpfdm;


struct tp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// GENERAL setup of one group: the block factors (given, or built from h
// and the reference pair of op), then P_d S_d = M_d S_d Lambda_d for every
// block and direction on host threads, the singularity check per block, and
// the upload of S and lambda (and of the factors of a length group, which
// the solve's residual needs).
static tp_status setup_general(Plan& plan, GroupInfo& g, int gi, int op, double tol) {
    if (g.nblocks == 0) return TP_OK;
    const int n = g.n;
    const size_t nn = static_cast<size_t>(n) * n;
    const size_t nbd = static_cast<size_t>(g.nblocks) * 3;
    std::vector<double> fac(nbd * 2 * nn);
    if (g.factors) {
        hipError_t e = hipMemcpy(fac.data(), g.fac, fac.size() * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_error(e, "readback of block factors");
    } else {
        std::vector<double> h(nbd);
        hipError_t e = hipMemcpy(h.data(), g.h, h.size() * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_error(e, "readback of h");
        const RefData& r = plan.ref[n];
        const double* Ph = op == TP_OP_CELL ? r.A : r.K;
        for (size_t bd = 0; bd < nbd; ++bd)
            for (size_t k = 0; k < nn; ++k) {
                fac[(2 * bd) * nn + k] = h[bd] * r.M[k];
                fac[(2 * bd + 1) * nn + k] = Ph[k] / h[bd];
            }
    }
    const size_t ne = nn + n;
    std::vector<double> eig(nbd * ne);
    std::vector<int64_t> bad_spd(16, INT64_MAX);
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&](unsigned t) {
        const size_t lo = nbd * t / nth, hi = nbd * (t + 1) / nth;
        std::vector<double> M(nn), P(nn);
        for (size_t bd = lo; bd < hi; ++bd) {
            const double* Fm = &fac[(2 * bd) * nn];
            const double* Fp = &fac[(2 * bd + 1) * nn];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    M[i * n + j] = 0.5 * (Fm[i * n + j] + Fm[j * n + i]);
                    P[i * n + j] = 0.5 * (Fp[i * n + j] + Fp[j * n + i]);
                }
            if (gen_eigen(n, M.data(), P.data(), &eig[bd * ne], &eig[bd * ne + nn]) != 0) {
                bad_spd[t] = static_cast<int64_t>(bd);
                return;
            }
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nth; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
    const int64_t bad = *std::min_element(bad_spd.begin(), bad_spd.end());
    if (bad != INT64_MAX)
        return set_error(TP_ERR_NOT_SPD, "group " + std::to_string(gi) + ": mass factor of block " +
                                             std::to_string(bad / 3) + " direction " + std::to_string(bad % 3) +
                                             " is not SPD");
    for (int64_t b = 0; b < g.nblocks; ++b) {
        double lo = 0.0, hi = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double* lam = &eig[(3 * b + d) * ne + nn];
            lo += lam[0];
            hi += lam[n - 1];
        }
        if (!(lo > tol * hi))
            return set_error(TP_ERR_SINGULAR, "group " + std::to_string(gi) + ": block " + std::to_string(b) +
                                                  " is singular: smallest/largest eigenvalue sum = " +
                                                  std::to_string(lo / hi));
    }
    tp_status st = TP_OK;
    if (!g.factors) st = upload_both(fac, &g.fac, &g.fac32, "block factors");
    if (st == TP_OK) st = upload_both(eig, &g.eig, &g.eig32, "block eigen-decompositions");
    return st;
}

// One group's call with the kernel family chosen by apply_kind & co.
static tp_status group_apply(const Plan& p, const GroupInfo& g, int op, const void* u, void* v, tp_dtype dt,
                             hipStream_t s) {
    const RefData& r = p.ref[g.n];
    switch (apply_kind(p, g, dt, u, v)) {
        case KIND_GENERAL: return launch_apply_gen(p, g, u, v, dt, s);
        case KIND_LANE: return launch_apply(p, g, op == TP_OP_CELL ? r.A : r.K, u, v, dt, s);
        case KIND_MFMA: return launch_apply_mfma(p, g, op, u, v, dt, s);
        default: return launch_apply_eo(p, g, op, u, v, dt, s);
    }
}
static tp_status group_inverse(const Plan& p, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                               hipStream_t s) {
    switch (inverse_kind(p, g, dt, r, x)) {
        case KIND_GENERAL: return launch_inverse_gen(p, g, r, x, dt, s);
        case KIND_LANE: return launch_inverse(p, g, r, x, dt, s);
        case KIND_MFMA: return launch_inverse_mfma(p, g, r, x, dt, s);
        default: return launch_inverse_eo(p, g, r, x, dt, s);
    }
}
static tp_status group_solve(const Plan& p, const GroupInfo& g, const double* b, double* x, tp_dtype inner,
                             double rtol, int maxit, int32_t* iters, double* relres, const SolveWork& w,
                             int64_t part_base, int64_t* nparts, hipStream_t s) {
    switch (solve_kind(p, g)) {
        case KIND_GENERAL:
            return launch_solve_gen(p, g, b, x, inner, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case KIND_LANE:
            return launch_solve_lane(p, g, b, x, inner, rtol, maxit, iters, relres, w, part_base, nparts, s);
        default: return launch_solve(p, g, b, x, inner, rtol, maxit, iters, relres, w, part_base, nparts, s);
    }
}

namespace {
tp_status hermite_reference(int n, RefData& r);
// Mesh plans in the Hermite-type basis with n >= 5 serve the coupled
// operator, PCG and the change of basis; their block calls are not built.
bool hermite_wave(const Plan& p) {
    return p.basis == TP_BASIS_HERMITE && !p.groups.empty() && p.groups[0].n > kLaneMaxN;
}
tp_status hermite_wave_error() {
    return set_error(TP_ERR_UNSUPPORTED,
                     "block calls on plans in the Hermite-type basis need n = 4 (n >= 5 serves the coupled operator)");
}
}

extern "C" {

const char* tp_last_error(void) { return g_last_error.c_str(); }

const char* tp_version(void) { return "tpfdm 0.1 (gfx950)"; }

void tp_plan_opts_default(tp_plan_opts* opts) {
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->penalty_C = 2.0;
    opts->persistent = 0;
}

tp_status tp_reference_matrices(int32_t n, double penalty_C, double* M, double* K, double* A) {
    if (n < kMinN || n > kMaxN) return set_error(TP_ERR_UNSUPPORTED, "n must be in [2, 8]");
    if (!(penalty_C > 0.0) || !std::isfinite(penalty_C))
        return set_error(TP_ERR_ARG, "penalty_C must be finite and > 0");
    reference_matrices(n, penalty_C, M, K, A);
    return TP_OK;
}

tp_status tp_reference_basis(int32_t n, int32_t basis, int32_t blocks, double penalty_C, double* M, double* K,
                             double* A, double* T) {
    if (n < kMinN || n > kMaxN) return set_error(TP_ERR_UNSUPPORTED, "n must be in [2, 8]");
    if (!(penalty_C > 0.0) || !std::isfinite(penalty_C))
        return set_error(TP_ERR_ARG, "penalty_C must be finite and > 0");
    if (basis != TP_BASIS_LAGRANGE && basis != TP_BASIS_HERMITE) return set_error(TP_ERR_ARG, "invalid basis");
    if (blocks != TP_BLOCKS_CELLS && blocks != TP_BLOCKS_PATCHES) return set_error(TP_ERR_ARG, "invalid blocks");
    if (basis == TP_BASIS_HERMITE && (n < 4 || blocks != TP_BLOCKS_CELLS))
        return set_error(TP_ERR_UNSUPPORTED, "the Hermite-type basis is supported for cells with n >= 4");
    if (blocks == TP_BLOCKS_PATCHES && (n % 2 != 0 || n < 4))
        return set_error(TP_ERR_UNSUPPORTED, "patch blocks have n = 2 (p+1) in {4, 6, 8}");
    RefData r;
    if (blocks == TP_BLOCKS_PATCHES)
        patch_reference(n / 2, penalty_C, r.M, r.K, r.A);
    else
        reference_matrices(n, penalty_C, r.M, r.K, r.A);
    endpoint_derivatives(n, r.g0, r.g1);
    prolongation_1d(n, r.P0, r.P1);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) r.T[i * n + j] = r.Ti[i * n + j] = i == j ? 1.0 : 0.0;
    if (basis == TP_BASIS_HERMITE) {
        tp_status st = hermite_reference(n, r);
        if (st != TP_OK) return st;
    }
    for (int i = 0; i < n * n; ++i) {
        if (M) M[i] = r.M[i];
        if (K) K[i] = r.K[i];
        if (A) A[i] = r.A[i];
        if (T) T[i] = r.T[i];
    }
    return TP_OK;
}

tp_status tp_reference_eigen(int32_t n, double penalty_C, tp_operator op, double* S, double* lam) {
    if (n < kMinN || n > kMaxN) return set_error(TP_ERR_UNSUPPORTED, "n must be in [2, 8]");
    if (!valid_op(op)) return set_error(TP_ERR_ARG, "invalid operator");
    if (!S || !lam) return set_error(TP_ERR_ARG, "S and lam must be non-null");
    if (!(penalty_C > 0.0) || !std::isfinite(penalty_C))
        return set_error(TP_ERR_ARG, "penalty_C must be finite and > 0");
    double M[kMaxN * kMaxN], K[kMaxN * kMaxN], A[kMaxN * kMaxN];
    reference_matrices(n, penalty_C, M, K, A);
    if (gen_eigen(n, M, op == TP_OP_CELL ? A : K, S, lam) != 0)
        return set_error(TP_ERR_NOT_SPD, "reference mass matrix is not SPD");
    return TP_OK;
}

}  // extern "C"

namespace {
tp_status plan_create(const tp_group* groups, int32_t ngroups, const tp_plan_opts* opts, int basis, tp_plan** out);

// Reference data of the Hermite-type basis from the Lagrange data already
// in r: the same bilinear forms in the new basis (M, K, A <- T^T X T), the
// endpoint derivatives g <- T^T g, the child embeddings P_c <- T^{-1} P_c T.
tp_status hermite_reference(int n, RefData& r) {
    hermite_transform(n, r.T);
    if (!invert_small(n, r.T, r.Ti)) return set_error(TP_ERR_NOT_SPD, "Hermite basis change is singular");
    congruence(n, r.T, r.M);
    congruence(n, r.T, r.K);
    congruence(n, r.T, r.A);
    double g0[kMaxN], g1[kMaxN];
    for (int j = 0; j < n; ++j) {
        g0[j] = g1[j] = 0.0;
        for (int i = 0; i < n; ++i) g0[j] += r.T[i * n + j] * r.g0[i], g1[j] += r.T[i * n + j] * r.g1[i];
    }
    for (int j = 0; j < n; ++j) r.g0[j] = g0[j], r.g1[j] = g1[j];
    for (double* P : {r.P0, r.P1}) {
        double Y[kMaxN * kMaxN];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += P[i * n + k] * r.T[k * n + j];
                Y[i * n + j] = s;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += r.Ti[i * n + k] * Y[k * n + j];
                P[i * n + j] = s;
            }
    }
    return TP_OK;
}
}  // namespace

extern "C" tp_status tp_plan_create(const tp_group* groups, int32_t ngroups, const tp_plan_opts* opts,
                                    tp_plan** out) {
    return plan_create(groups, ngroups, opts, TP_BASIS_LAGRANGE, out);
}

namespace {
tp_status plan_create(const tp_group* groups, int32_t ngroups, const tp_plan_opts* opts, int basis, tp_plan** out) {
    if (!out) return set_error(TP_ERR_ARG, "out must be non-null");
    *out = nullptr;
    if (ngroups < 0 || (ngroups > 0 && !groups)) return set_error(TP_ERR_ARG, "invalid group array");
    tp_plan_opts o;
    tp_plan_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.penalty_C > 0.0) || !std::isfinite(o.penalty_C))
        return set_error(TP_ERR_ARG, "penalty_C must be finite and > 0");
    for (int i = 0; i < 5; ++i)
        if (o.reserved[i] != 0) return set_error(TP_ERR_ARG, "reserved option fields must be zero");
    if (o.blocks != TP_BLOCKS_CELLS && o.blocks != TP_BLOCKS_PATCHES) return set_error(TP_ERR_ARG, "invalid blocks");
    if (o.blocks == TP_BLOCKS_PATCHES)
        for (int gi = 0; gi < ngroups; ++gi) {
            if (groups[gi].n % 2 != 0 || groups[gi].n < 4)
                return set_error(TP_ERR_UNSUPPORTED,
                                 "group " + std::to_string(gi) + ": patch blocks have n = 2 (p+1) in {4, 6, 8}");
            if (groups[gi].M)
                return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": patch groups are given by h");
        }
    if (o.mapping < TP_MAP_AUTO || o.mapping > TP_MAP_WAVE) return set_error(TP_ERR_ARG, "invalid mapping");
    if (basis == TP_BASIS_HERMITE) {
        // degree p >= 3; n = 4 runs the lane kernels, n >= 5 the wave kernels
        for (int gi = 0; gi < ngroups; ++gi)
            if (groups[gi].n < 4)
                return set_error(TP_ERR_UNSUPPORTED, "the Hermite-type basis needs n >= 4 (p >= 3)");
        if (o.mapping == TP_MAP_WAVE && ngroups > 0 && groups[0].n == 4)
            return set_error(TP_ERR_UNSUPPORTED, "the Hermite-type basis of n = 4 runs on the lane mapping");
    }

    // validate groups and their element ranges
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int gi = 0; gi < ngroups; ++gi) {
        const tp_group& g = groups[gi];
        if (g.n < kMinN || g.n > kMaxN)
            return set_error(TP_ERR_UNSUPPORTED, "group " + std::to_string(gi) + ": n must be in [2, 8]");
        if (!is_pow2(g.layout_B) || g.layout_B > 1024)
            return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": layout_B must be a power of two <= 1024");
        if (g.nblocks < 0 || g.nblocks > (int64_t(1) << 31) - 1)
            return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": nblocks out of range");
        if (g.offset < 0) return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": negative offset");
        if ((g.M == nullptr) != (g.P == nullptr))
            return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": M and P must be given together");
        if (g.M && g.h)
            return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": a factor group takes no h");
        if (g.M && o.persistent)
            return set_error(TP_ERR_UNSUPPORTED, "group " + std::to_string(gi) +
                                                     ": factor groups are not supported by persistent plans");
        if (g.nblocks > 0 && !g.h && !g.M)
            return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": h is null");
        const int64_t n3 = int64_t(g.n) * g.n * g.n;
        const int64_t tiles = (g.nblocks + g.layout_B - 1) / g.layout_B;
        const int64_t elems = tiles * n3 * g.layout_B;
        if (elems > 0) ranges.push_back({g.offset, g.offset + elems});
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second)
            return set_error(TP_ERR_ARG, "group element ranges overlap");

    tp_plan* p = new (std::nothrow) tp_plan();
    if (!p) return set_error(TP_ERR_OOM, "host allocation failed");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_error(e, "hipGetDevice");
    }
    p->penalty_C = o.penalty_C;
    p->basis = basis;
    p->patches = o.blocks == TP_BLOCKS_PATCHES;
    p->persistent = o.persistent != 0;
    p->mapping = o.mapping;
    int64_t canon = 0, block0 = 0;
    std::vector<double> hbuf;
    for (int gi = 0; gi < ngroups; ++gi) {
        const tp_group& g = groups[gi];
        GroupInfo info;
        info.n = g.n;
        info.logB = ilog2(g.layout_B);
        info.nblocks = g.nblocks;
        info.offset = g.offset;
        info.canon = canon;
        info.block0 = block0;
        info.h = nullptr;
        const int64_t n3 = int64_t(g.n) * g.n * g.n;
        canon += g.nblocks * n3;
        block0 += g.nblocks;
        const int64_t tiles = (g.nblocks + g.layout_B - 1) / g.layout_B;
        p->vec_elems = std::max(p->vec_elems, g.offset + tiles * n3 * g.layout_B);
        info.factors = g.M != nullptr;
        p->groups.push_back(info);
        if (g.nblocks == 0) continue;
        if (info.factors) {
            tp_status st = copy_factors(p->groups.back(), g.M, g.P, gi);
            if (st != TP_OK) {
                free_plan_memory(p);
                delete p;
                return st;
            }
            continue;
        }
        // stage h on the host to validate it, then copy to plan-owned memory
        hbuf.resize(static_cast<size_t>(g.nblocks) * 3);
        e = hipMemcpy(hbuf.data(), g.h, hbuf.size() * sizeof(double), hipMemcpyDefault);
        if (e != hipSuccess) {
            free_plan_memory(p);
            delete p;
            return hip_error(e, "copy of h");
        }
        for (size_t i = 0; i < hbuf.size(); ++i)
            if (!(hbuf[i] > 0.0) || !std::isfinite(hbuf[i])) {
                free_plan_memory(p);
                delete p;
                return set_error(TP_ERR_ARG, "group " + std::to_string(gi) + ": h must be finite and > 0 (block " +
                                                 std::to_string(i / 3) + ")");
            }
        tp_status st = alloc_dev(reinterpret_cast<void**>(&p->groups.back().h), hbuf.size() * sizeof(double), "h");
        if (st != TP_OK) {
            free_plan_memory(p);
            delete p;
            return st;
        }
        e = hipMemcpy(p->groups.back().h, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_plan_memory(p);
            delete p;
            return hip_error(e, "copy of h");
        }
    }
    p->ndof = canon;
    p->nblocks = block0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
        p->wave_grid = static_cast<int64_t>(cus) * 8, p->cus = cus;
    // The lane solve runs one wave (64 blocks) per SIMD; below one tile per
    // SIMD the wave-per-tile solve spreads a group over more waves (AUTO).
    // TP_MAP_LANE asks for the lane solve at any size.
    for (auto& g : p->groups)
        g.lane_solve = use_lane(*p, g) && (p->mapping == TP_MAP_LANE || p->basis == TP_BASIS_HERMITE ||
                                           (g.nblocks + 63) / 64 >= static_cast<int64_t>(p->cus) * 4);
    tp_status st = alloc_dev(&p->summary_dev, sizeof(SolveSummary), "solve summary");
    if (st == TP_OK) {
        hipError_t he = hipHostMalloc(&p->summary_host, sizeof(SolveSummary),
                                      hipHostMallocMapped | hipHostMallocCoherent);
        if (he != hipSuccess) p->summary_host = nullptr, st = hip_error(he, "pinned solve summary");
        if (st == TP_OK) {
            he = hipHostGetDevicePointer(&p->summary_host_dev, p->summary_host, 0);
            if (he != hipSuccess) st = hip_error(he, "pinned solve summary (device address)");
        }
    }
    p->partials_cap = static_cast<int64_t>(p->groups.size() + 1) * p->cus * kMaxWgPerCu;
    if (st == TP_OK)
        st = alloc_dev(&p->partials_dev, static_cast<size_t>(p->partials_cap) * sizeof(SolvePartial), "solve partials");
    if (st == TP_OK)
        st = alloc_dev(&p->eo_dev, static_cast<size_t>(kMaxN + 1) * EO_NTAB * 2 * kEOSlot * sizeof(double),
                       "even-odd tables");
    for (auto& g : p->groups) {
        if (st != TP_OK) break;
        RefData& r = p->ref[g.n];
        if (r.built) continue;
        if (p->patches)
            patch_reference(g.n / 2, p->penalty_C, r.M, r.K, r.A);
        else
            reference_matrices(g.n, p->penalty_C, r.M, r.K, r.A);
        endpoint_derivatives(g.n, r.g0, r.g1);
        prolongation_1d(g.n, r.P0, r.P1);
        for (int i = 0; i < g.n; ++i)
            for (int j = 0; j < g.n; ++j) r.T[i * g.n + j] = r.Ti[i * g.n + j] = i == j ? 1.0 : 0.0;
        r.built = true;
        double tab[kEOSlot];
        if (p->basis == TP_BASIS_HERMITE) {
            st = hermite_reference(g.n, r);
            if (st != TP_OK) break;
            if (g.n > kLaneMaxN) {
                // the wave kernels work on the coefficients with the sign of
                // the derivative-at-1 function flipped, where the matrices
                // are centrosymmetric: tables of D X D, D = diag(hermite_sign)
                const int hc = (g.n + 1) / 2, h = g.n / 2;
                const int cnt = 2 * (hc * hc + h * h);
                double Mf[kMaxN * kMaxN], Kf[kMaxN * kMaxN], Af[kMaxN * kMaxN], Ff[kMaxN * kMaxN];
                for (int i = 0; i < g.n; ++i)
                    for (int j = 0; j < g.n; ++j) {
                        const double sg = hermite_sign(g.n, i) * hermite_sign(g.n, j);
                        Mf[i * g.n + j] = sg * r.M[i * g.n + j];
                        Kf[i * g.n + j] = sg * r.K[i * g.n + j];
                        Af[i * g.n + j] = sg * r.A[i * g.n + j];
                        Ff[i * g.n + j] = Af[i * g.n + j] - Kf[i * g.n + j];
                    }
                const double* P3[3] = {Kf, Af, Ff};
                const int slot[3] = {EO_APPLY_K, EO_APPLY_A, EO_APPLY_F};
                for (int t = 0; t < 3 && st == TP_OK; ++t) {
                    if (!build_eo_apply(g.n, Mf, P3[t], tab)) {
                        st = set_error(TP_ERR_UNSUPPORTED, "sign-flipped Hermite matrices are not centrosymmetric");
                        break;
                    }
                    st = upload_eo(*p, g.n, slot[t], tab, cnt);
                }
                continue;
            }
            const int n2 = g.n * g.n;
            for (int i = 0; i < n2; ++i) tab[i] = r.M[i], tab[n2 + i] = r.K[i];
            st = upload_eo(*p, g.n, EO_PLAIN_K, tab, 2 * n2);
            if (st != TP_OK) break;
            for (int i = 0; i < n2; ++i) tab[n2 + i] = r.A[i];
            st = upload_eo(*p, g.n, EO_PLAIN_A, tab, 2 * n2);
            continue;
        }
        const int hc = (g.n + 1) / 2, h = g.n / 2;
        const int cnt = 2 * (hc * hc + h * h);
        if (!build_eo_apply(g.n, r.M, r.K, tab)) {
            st = set_error(TP_ERR_UNSUPPORTED, "reference matrices are not centrosymmetric");
            break;
        }
        st = upload_eo(*p, g.n, EO_APPLY_K, tab, cnt);
        if (st != TP_OK) break;
        if (!build_eo_apply(g.n, r.M, r.A, tab)) {
            st = set_error(TP_ERR_UNSUPPORTED, "reference matrices are not centrosymmetric");
            break;
        }
        st = upload_eo(*p, g.n, EO_APPLY_A, tab, cnt);
        if (st != TP_OK) break;
        double F[kMaxN * kMaxN];
        for (int i = 0; i < g.n * g.n; ++i) F[i] = r.A[i] - r.K[i];
        if (!build_eo_apply(g.n, r.M, F, tab)) {
            st = set_error(TP_ERR_UNSUPPORTED, "reference matrices are not centrosymmetric");
            break;
        }
        st = upload_eo(*p, g.n, EO_APPLY_F, tab, cnt);
        if (st != TP_OK || g.n > kLaneMaxN) continue;
        // plain factors for the lane-per-block kernels (2 n^2 <= kEOSlot for n <= 4)
        const int n2 = g.n * g.n;
        static_assert(2 * kLaneMaxN * kLaneMaxN <= kEOSlot, "plain tables exceed a slot");
        for (int i = 0; i < n2; ++i) tab[i] = r.M[i], tab[n2 + i] = r.K[i];
        st = upload_eo(*p, g.n, EO_PLAIN_K, tab, 2 * n2);
        if (st != TP_OK) break;
        for (int i = 0; i < n2; ++i) tab[n2 + i] = r.A[i];
        st = upload_eo(*p, g.n, EO_PLAIN_A, tab, 2 * n2);
    }
    if (st == TP_OK) st = persistent_setup(*p);
    if (st == TP_OK && p->ref[8].built && p->basis != TP_BASIS_HERMITE) {  // MFMA operand tables of n = 8
        const RefData& r8 = p->ref[8];
        for (int op = 0; op < 2 && st == TP_OK; ++op)
            for (int et = 0; et < 2 && st == TP_OK; ++et) {
                std::vector<uint16_t> tabv;
                build_mfma_tables(r8.M, op == 1 ? r8.A : r8.K, nullptr, nullptr, et == 1, &tabv, nullptr);
                st = alloc_dev(&p->mfma_apply_dev[op][et], tabv.size() * 2, "MFMA tables");
                if (st == TP_OK) {
                    hipError_t he = hipMemcpy(p->mfma_apply_dev[op][et], tabv.data(), tabv.size() * 2,
                                              hipMemcpyHostToDevice);
                    if (he != hipSuccess) st = hip_error(he, "MFMA table upload");
                }
            }
    }
    if (st != TP_OK) {
        free_plan_memory(p);
        delete p;
        return st;
    }
    *out = p;
    return TP_OK;
}
}  // namespace


namespace tpfdm {
// The block-local solve of tp_solve and tp_solve_static: the launches write
// their partial summaries to w.parts and the reduction the summary to
// w.summary.
tp_status solve_impl(tp_plan* plan, const double* b, double* x, tp_dtype inner, double rtol, int32_t maxit,
                     int32_t* iters, double* relres, tp_solve_summary* summary, hipStream_t stream,
                     const SolveWork& w) {
    if (hermite_wave(*plan)) return hermite_wave_error();
    if (plan->inverse_op < 0 || (plan->factor_mode == TP_FACTOR_SCALED && plan->inverse_op != TP_OP_CELL))
        return set_error(TP_ERR_STATE, "tp_solve needs tp_setup_inverse(TP_OP_CELL) first");
    if (inner != TP_F64 && inner != TP_F32 && inner != TP_F16 && inner != TP_BF16)
        return set_error(TP_ERR_ARG, "invalid inner precision");
    if (!(rtol >= 0.0) || !std::isfinite(rtol)) return set_error(TP_ERR_ARG, "rtol must be finite and >= 0");
    if (maxit < 0) return set_error(TP_ERR_ARG, "maxit must be >= 0");
    if (plan->vec_elems > 0 && (!b || !x)) return set_error(TP_ERR_ARG, "b and x must be non-null");
    if (static_cast<const void*>(b) == static_cast<const void*>(x) && b)
        return set_error(TP_ERR_ARG, "b and x must not alias");
    tp_status st = TP_OK;
    int64_t nparts = 0;
    if (plan->persistent) {
        st = launch_solve_persistent(*plan, b, x, inner, rtol, maxit, iters, relres, w, &nparts, stream);
        if (st != TP_OK) return st;
    } else {
        for (size_t i = 0; st == TP_OK && i < plan->groups.size(); ++i) {
            const GroupInfo& g = plan->groups[i];
                int64_t np = 0;
            st = group_solve(*plan, g, b, x, inner, rtol, maxit, iters, relres, w, nparts, &np, stream);
            nparts += np;
        }
        if (st != TP_OK) return st;
    }
    // With a summary requested and the plan's own workspace, the reduction
    // also writes the summary into pinned host memory, tagged with this
    // call's sequence number, so the readback is only the stream's
    // synchronization (a device-to-host copy of the 24 bytes added 5-8 us
    // per call).  A tag that does not match falls back to the copy.
    int tag = 0;
    if (summary && w.host && plan->summary_host) {
        plan->summary_seq = plan->summary_seq % 1000000000 + 1;
        tag = plan->summary_seq;
    }
    st = launch_summary_reduce(w, nparts, tag ? w.host : nullptr, tag, stream);
    if (st != TP_OK) return st;
    if (summary) {
        SolveSummary hs{};
        hipError_t e = hipStreamSynchronize(stream);
        if (e == hipSuccess && tag) std::memcpy(&hs, plan->summary_host, sizeof(hs));
        if (e == hipSuccess && (!tag || hs.pad != tag)) {
            e = hipMemcpyAsync(&hs, w.summary, sizeof(hs), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
        }
        if (e != hipSuccess) return hip_error(e, "solve summary readback");
        summary->max_iters = hs.max_iters;
        summary->n_failed = hs.n_failed;
        double mr;
        std::memcpy(&mr, &hs.max_relres_bits, sizeof(mr));
        summary->max_relres = mr;
        if (hs.nonfinite > 0)
            return set_error(TP_ERR_NONFINITE, std::to_string(hs.nonfinite) + " blocks had a non-finite residual");
        if (hs.n_failed > 0)
            return set_error(TP_ERR_NOT_CONVERGED, std::to_string(hs.n_failed) + " blocks missed rtol");
    }
    return TP_OK;
}

// Upper bound on the per-workgroup partial summaries one solve of the plan
// writes: every solve launch runs at most one workgroup per tile and at
// most kMaxWgPerCu resident workgroups per compute unit.
int64_t solve_parts_bound(const Plan& p) {
    const int64_t per_launch = static_cast<int64_t>(p.cus) * kMaxWgPerCu;
    if (p.persistent) return per_launch;
    int64_t total = 0;
    for (const auto& g : p.groups) {
        const int bpw = g.n * g.n >= 64 ? 1 : 64 / (g.n * g.n);
        const int64_t tiles = std::max<int64_t>((g.nblocks + 63) / 64, (g.nblocks + bpw - 1) / bpw);
        total += std::min(tiles, per_launch);
    }
    return total;
}

}  // namespace tpfdm

namespace tpfdm {
namespace {

// Scratch vectors and timing of the autotuner: nsets pairs (U, V) of
// plan-sized buffers of pseudo-random values, rotated so that one pass
// streams from HBM rather than from the last-level cache, and, for the
// solve, an FP64 right-hand side and iterate.
struct TuneBench {
    Plan* plan = nullptr;
    int nsets = 1;
    void* U[8] = {};
    void* V[8] = {};
    void *b = nullptr, *x = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int cur = 0;
    int reps = 10;

    tp_status init(Plan* p, tp_dtype dt, bool solve, int r) {
        plan = p;
        reps = r;
        const size_t es = static_cast<size_t>(esize_of(dt));
        const size_t ne = static_cast<size_t>(p->vec_elems);
        const size_t pair_bytes = 2 * ne * es;
        nsets = static_cast<int>(std::max<size_t>(1, std::min<size_t>(8, (768u << 20) / pair_bytes + 1)));
        tp_status st = TP_OK;
        for (int k = 0; st == TP_OK && k < nsets; ++k) {
            st = alloc_dev(&U[k], ne * es, "autotune scratch");
            if (st == TP_OK) st = alloc_dev(&V[k], ne * es, "autotune scratch");
        }
        if (st == TP_OK && solve) st = alloc_dev(&b, ne * sizeof(double), "autotune scratch");
        if (st == TP_OK && solve) st = alloc_dev(&x, ne * sizeof(double), "autotune scratch");
        hipError_t e = hipSuccess;
        if (st == TP_OK) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (st == TP_OK && e == hipSuccess) e = hipEventCreate(&e0);
        if (st == TP_OK && e == hipSuccess) e = hipEventCreate(&e1);
        if (st == TP_OK && e != hipSuccess) st = hip_error(e, "autotune stream");
        for (int k = 0; st == TP_OK && k < nsets; ++k)
            st = launch_fill(U[k], static_cast<int64_t>(ne), dt, 1, false, s);
        if (st == TP_OK && solve) st = launch_fill(b, static_cast<int64_t>(ne), TP_F64, 2, false, s);
        if (st == TP_OK) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_error(e, "autotune scratch fill");
        }
        return st;
    }
    // average microseconds of reps launches of f (after one warm-up); the
    // stream is idle again on return
    template <typename F>
    tp_status time(F f, double* out) {
        tp_status r = f();
        for (int i = 0; r == TP_OK && i < reps; ++i) {
            if (i == 0) {
                hipError_t he = hipEventRecord(e0, s);
                if (he != hipSuccess) return hip_error(he, "autotune event");
            }
            r = f();
        }
        if (r != TP_OK) return r;
        hipError_t he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) return hip_error(he, "autotune timing");
        *out = 1e3 * ms / reps;
        return TP_OK;
    }
    ~TuneBench() {
        if (s) (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        for (int k = 0; k < nsets; ++k) {
            if (U[k]) (void)hipFree(U[k]);
            if (V[k]) (void)hipFree(V[k]);
        }
        for (void* ptr : {b, x})
            if (ptr) (void)hipFree(ptr);
    }
};

// Tunes the single launch of a persistent plan for one call and dtype by
// coordinate descent over its parameters: per group (in turn) the tile body
// and the tiles per workgroup, then the segment order, then (solve) the
// grid.  Each candidate is uploaded and timed as the whole launch; the best
// of each step is kept.  A last comparison against the default
// configuration (best of three alternating timings each) guards against a
// choice that only won by noise.
tp_status tune_persistent_call(Plan& plan, int call, tp_dtype dt, TuneBench& tb, double* best_us) {
    PersistCfg& c = plan.pcfg[call][dt];
    const size_t ng = plan.groups.size();
    auto launch = [&]() -> tp_status {
        tb.cur = (tb.cur + 1) % tb.nsets;
        switch (call) {
            case PCALL_APPLY:
                return launch_apply_persistent(plan, TP_OP_NEUMANN, tb.U[tb.cur], tb.V[tb.cur], dt, tb.s);
            case PCALL_INVERSE: return launch_inverse_persistent(plan, tb.U[tb.cur], tb.V[tb.cur], dt, tb.s);
            default: {
                int64_t np = 0;
                tp_status r = launch_fill(tb.x, plan.vec_elems, TP_F64, 0, true, tb.s);
                if (r == TP_OK)
                    r = launch_solve_persistent(plan, static_cast<const double*>(tb.b), static_cast<double*>(tb.x),
                                                dt, 1e-10, 20, nullptr, nullptr, plan_work(plan), &np, tb.s);
                return r;
            }
        }
    };
    auto measure = [&](double* t) -> tp_status {
        tp_status r = persistent_upload(plan, call, dt);   // the stream is idle between timings
        if (r == TP_OK) r = tb.time(launch, t);
        return r;
    };
    const PersistCfg dflt = c;
    double best = 0.0;
    tp_status st = measure(&best);
    // per group: body and tiles per workgroup
    for (size_t gi = 0; st == TP_OK && gi < ng; ++gi) {
        const GroupInfo& g = plan.groups[gi];
        if (g.nblocks == 0) continue;
        const int8_t keep_lane = c.lane[gi], keep_tpw = c.tpw[gi];
        int8_t best_lane = keep_lane, best_tpw = keep_tpw;
        for (int lane = 0; st == TP_OK && lane < 2; ++lane) {
            if (lane && (call == PCALL_SOLVE || !persistent_lane_ok(plan, g))) continue;
            for (int8_t tpw : {int8_t(1), int8_t(2), int8_t(4), int8_t(8)}) {
                if (lane == keep_lane && tpw == keep_tpw) continue;
                c.lane[gi] = static_cast<int8_t>(lane);
                c.tpw[gi] = tpw;
                double t = 0.0;
                st = measure(&t);
                if (st != TP_OK) break;
                if (t < best) best = t, best_lane = c.lane[gi], best_tpw = tpw;
            }
        }
        c.lane[gi] = best_lane;
        c.tpw[gi] = best_tpw;
    }
    // segment order: as given, reversed, by degree descending and ascending
    if (st == TP_OK && ng > 1) {
        std::vector<std::vector<int32_t>> orders;
        std::vector<int32_t> o = c.order;
        std::reverse(o.begin(), o.end());
        orders.push_back(o);
        o = c.order;
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return plan.groups[a].n > plan.groups[b].n; });
        orders.push_back(o);
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return plan.groups[a].n < plan.groups[b].n; });
        orders.push_back(o);
        std::vector<int32_t> best_order = c.order;
        for (const auto& cand : orders) {
            if (cand == best_order) continue;
            c.order = cand;
            double t = 0.0;
            st = measure(&t);
            if (st != TP_OK) break;
            if (t < best) best = t, best_order = cand;
        }
        c.order = best_order;
    }
    // solve grid: occupancy grid, half of it, one workgroup per item
    if (st == TP_OK && call == PCALL_SOLVE) {
        int8_t best_grid = c.grid;
        for (int8_t gr : {int8_t(1), int8_t(2), int8_t(0)}) {
            if (gr == best_grid) continue;
            c.grid = gr;
            if (persistent_upload(plan, call, dt) == TP_OK && gr == 0 && c.items > plan.partials_cap) continue;
            double t = 0.0;
            st = measure(&t);
            if (st != TP_OK) break;
            if (t < best) best = t, best_grid = gr;
        }
        c.grid = best_grid;
    }
    if (st == TP_OK) {
        const PersistCfg tuned = c;
        double tt = 1e300, td = 1e300;
        for (int k = 0; st == TP_OK && k < 3; ++k) {
            double t = 0.0;
            c = dflt;
            st = measure(&t);
            td = std::min(td, t);
            if (st != TP_OK) break;
            c = tuned;
            st = measure(&t);
            tt = std::min(tt, t);
        }
        if (st == TP_OK && td <= tt) c = dflt, best = td;
        else best = tt;
        c.tuned = true;
    }
    if (st == TP_OK) st = persistent_upload(plan, call, dt);
    if (st != TP_OK) {                 // leave the plan in its default state
        c = dflt;
        (void)persistent_upload(plan, call, dt);
    }
    *best_us = best;
    return st;
}

tp_status autotune_persistent(Plan* plan, tp_dtype dtype, int reps, double* us) {
    if (reps <= 0) reps = 10;
    reps = std::max(reps, 30);       // single launches of a few microseconds need more samples
    const size_t ng = plan->groups.size();
    if (us)
        for (size_t i = 0; i < 3 * ng; ++i) us[i] = -1.0;
    if (plan->vec_elems == 0 || plan->nblocks == 0) return TP_OK;
    const bool inv = plan->inverse_op >= 0 && plan->factor_mode == TP_FACTOR_SCALED;
    const bool solve = inv && plan->inverse_op == TP_OP_CELL;
    TuneBench tb;
    tp_status st = tb.init(plan, dtype, solve, reps);
    for (int call = 0; st == TP_OK && call < 3; ++call) {
        if ((call == PCALL_INVERSE && !inv) || (call == PCALL_SOLVE && !solve)) continue;
        double t = -1.0;
        st = tune_persistent_call(*plan, call, dtype, tb, &t);
        if (st == TP_OK && us) us[call] = t;
    }
    return st;
}

}  // namespace
}  // namespace tpfdm

extern "C" {

tp_status tp_plan_destroy(tp_plan* plan) {
    if (!plan) return TP_OK;
    free_plan_memory(plan);
    delete plan;
    return TP_OK;
}

tp_status tp_plan_create_mesh(const tp_mesh* mesh, const tp_plan_opts* opts, tp_plan** out) {
    if (!out) return set_error(TP_ERR_ARG, "out must be non-null");
    *out = nullptr;
    if (!mesh) return set_error(TP_ERR_ARG, "mesh must be non-null");
    if (mesh->basis != TP_BASIS_LAGRANGE && mesh->basis != TP_BASIS_HERMITE)
        return set_error(TP_ERR_ARG, "invalid basis");
    if (opts && opts->blocks != TP_BLOCKS_CELLS) return set_error(TP_ERR_UNSUPPORTED, "mesh plans hold cells");
    if (opts && opts->persistent) return set_error(TP_ERR_UNSUPPORTED, "mesh plans cannot be persistent");
    int64_t ncells = 1;
    for (int d = 0; d < 3; ++d) {
        if (mesh->cells[d] < 1) return set_error(TP_ERR_ARG, "mesh cells must be >= 1 in every direction");
        if (!(mesh->h[d] > 0.0) || !std::isfinite(mesh->h[d]))
            return set_error(TP_ERR_ARG, "mesh h must be finite and > 0");
        ncells *= mesh->cells[d];
        if (ncells > (int64_t(1) << 31) - 1) return set_error(TP_ERR_ARG, "mesh has too many cells");
    }
    std::vector<double> h(static_cast<size_t>(ncells) * 3);
    for (int64_t c = 0; c < ncells; ++c)
        for (int d = 0; d < 3; ++d) h[c * 3 + d] = mesh->h[d];
    tp_group g;
    g.n = mesh->n;
    g.layout_B = mesh->layout_B;
    g.nblocks = ncells;
    g.h = h.data();
    g.offset = 0;
    g.M = nullptr;
    g.P = nullptr;
    tp_plan* p = nullptr;
    tp_status st = plan_create(&g, 1, opts, mesh->basis, &p);
    if (st != TP_OK) return st;
    p->mesh = true;
    for (int d = 0; d < 3; ++d) {
        p->mesh_m[d] = mesh->cells[d];
        p->mesh_h[d] = mesh->h[d];
    }
    *out = p;
    return TP_OK;
}

int64_t tp_plan_vector_elems(const tp_plan* plan) { return plan ? plan->vec_elems : -1; }
int64_t tp_plan_ndof(const tp_plan* plan) { return plan ? plan->ndof : -1; }
int64_t tp_plan_nblocks(const tp_plan* plan) { return plan ? plan->nblocks : -1; }

tp_status tp_apply(tp_plan* plan, tp_operator op, const void* u, void* v, tp_dtype dtype, hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!valid_op(op) && !coupled_op(op)) return set_error(TP_ERR_ARG, "invalid operator");
    if (!valid_dtype(dtype)) return set_error(TP_ERR_UNSUPPORTED, "invalid dtype");
    if (plan->vec_elems > 0 && (!u || !v)) return set_error(TP_ERR_ARG, "u and v must be non-null");
    if (u == v && u) return set_error(TP_ERR_ARG, "u and v must not alias");
    if (coupled_op(op)) {
        if (!plan->mesh) return set_error(TP_ERR_UNSUPPORTED, "the coupled SIPG operator needs a mesh plan");
        return launch_sipg(*plan, plan->groups[0], op == TP_OP_SIPG_FACE, u, v, dtype, stream);
    }
    if (hermite_wave(*plan)) return hermite_wave_error();
    if (plan->persistent) return launch_apply_persistent(*plan, op, u, v, dtype, stream);
    tp_status st = TP_OK;
    for (size_t i = 0; st == TP_OK && i < plan->groups.size(); ++i) {
        st = group_apply(*plan, plan->groups[i], op, u, v, dtype, stream);
    }
    return st;
}

tp_status tp_setup_inverse(tp_plan* plan, tp_operator op, tp_factor_mode mode, double singular_tol) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!valid_op(op)) return set_error(TP_ERR_ARG, "invalid operator");
    if (mode != TP_FACTOR_SCALED && mode != TP_FACTOR_GENERAL) return set_error(TP_ERR_ARG, "invalid factor mode");
    if (!(singular_tol > 0.0)) singular_tol = 1e-12;
    plan->inverse_op = -1;
    for (auto& g : plan->groups) free_block_factors(g, false);
    if (mode == TP_FACTOR_GENERAL) {
        if (plan->persistent) return set_error(TP_ERR_UNSUPPORTED, "persistent plans support TP_FACTOR_SCALED only");
        for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
            tp_status st = setup_general(*plan, plan->groups[gi], static_cast<int>(gi), op, singular_tol);
            if (st != TP_OK) {
                for (auto& g : plan->groups) free_block_factors(g, false);
                return st;
            }
        }
        plan->factor_mode = TP_FACTOR_GENERAL;
        plan->inverse_op = op;
        return TP_OK;
    }
    for (const auto& g : plan->groups)
        if (g.factors)
            return set_error(TP_ERR_UNSUPPORTED, "groups given by block factors need TP_FACTOR_GENERAL");
    plan->factor_mode = TP_FACTOR_SCALED;
    for (int n = kMinN; n <= kMaxN; ++n) {
        RefData& r = plan->ref[n];
        r.eig_ready = false;
        if (!r.built) continue;
        if (gen_eigen(n, r.M, op == TP_OP_CELL ? r.A : r.K, r.S, r.lam) != 0)
            return set_error(TP_ERR_NOT_SPD, "reference mass matrix of n=" + std::to_string(n) + " is not SPD");
        // eigenvalue sums lam_i s_x + lam_j s_y + lam_k s_z of any block are
        // bounded below by lam_min (s_x + s_y + s_z) and above by lam_max (...)
        if (!(r.lam[0] > singular_tol * r.lam[n - 1]))
            return set_error(TP_ERR_SINGULAR, "operator of n=" + std::to_string(n) +
                                                  " is singular: lambda_min/lambda_max = " +
                                                  std::to_string(r.lam[0] / r.lam[n - 1]));
        double tab[kEOSlot];
        const int cnt = ((n + 1) / 2) * ((n + 1) / 2) + (n / 2) * (n / 2) + n;
        tp_status st = TP_OK;
        if (plan->basis != TP_BASIS_HERMITE || n > kLaneMaxN) {   // the lane kernels use plain factors
            // Hermite-type basis: eigenvectors of the sign-flipped pair (D S)
            double Sf[kMaxN * kMaxN];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    Sf[i * n + j] = (plan->basis == TP_BASIS_HERMITE ? hermite_sign(n, i) : 1.0) * r.S[i * n + j];
            if (!build_eo_inverse(n, Sf, r.lam, tab))
                return set_error(TP_ERR_UNSUPPORTED, "eigenvectors of n=" + std::to_string(n) +
                                                         " are not split into symmetric and antisymmetric ones");
            st = upload_eo(*plan, n, EO_INV, tab, cnt);
            if (st != TP_OK) return st;
        }
        if (n <= kLaneMaxN) {  // plain factors for the lane-per-block kernels
            static_assert(kLaneMaxN * kLaneMaxN + kLaneMaxN <= kEOSlot, "plain tables exceed a slot");
            for (int i = 0; i < n * n; ++i) tab[i] = r.S[i];
            for (int i = 0; i < n; ++i) tab[n * n + i] = r.lam[i];
            st = upload_eo(*plan, n, EO_PLAIN_S, tab, n * n + n);
            if (st != TP_OK) return st;
        }
        if (n == 8 && plan->basis != TP_BASIS_HERMITE) {  // MFMA operand tables of the inverse
            for (int et = 0; et < 2; ++et) {
                std::vector<uint8_t> tabv;
                build_mfma_tables(r.M, r.A, r.S, r.lam, et == 1, nullptr, &tabv);
                if (!plan->mfma_inv_dev[et]) {
                    st = alloc_dev(&plan->mfma_inv_dev[et], tabv.size(), "MFMA tables");
                    if (st != TP_OK) return st;
                }
                hipError_t he = hipMemcpy(plan->mfma_inv_dev[et], tabv.data(), tabv.size(), hipMemcpyHostToDevice);
                if (he != hipSuccess) return hip_error(he, "MFMA table upload");
            }
        }
        r.eig_ready = true;
    }
    plan->inverse_op = op;
    return TP_OK;
}

tp_status tp_apply_inverse(tp_plan* plan, const void* r, void* x, tp_dtype dtype, hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (hermite_wave(*plan)) return hermite_wave_error();
    if (!valid_dtype(dtype)) return set_error(TP_ERR_UNSUPPORTED, "invalid dtype");
    if (plan->inverse_op < 0) return set_error(TP_ERR_STATE, "tp_setup_inverse has not succeeded on this plan");
    if (plan->vec_elems > 0 && (!r || !x)) return set_error(TP_ERR_ARG, "r and x must be non-null");
    if (r == x && r) return set_error(TP_ERR_ARG, "r and x must not alias");
    if (plan->persistent) return launch_inverse_persistent(*plan, r, x, dtype, stream);
    tp_status st = TP_OK;
    for (size_t i = 0; st == TP_OK && i < plan->groups.size(); ++i) {
        st = group_inverse(*plan, plan->groups[i], r, x, dtype, stream);
    }
    return st;
}

tp_status tp_solve(tp_plan* plan, const double* b, double* x, tp_dtype inner, double rtol, int32_t maxit,
                   int32_t* iters, double* relres, tp_solve_summary* summary, hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    return solve_impl(plan, b, x, inner, rtol, maxit, iters, relres, summary, stream, plan_work(*plan));
}

tp_status tp_solve_static(tp_plan* plan, const double* b, double* x, tp_dtype inner, double rtol, int32_t maxit,
                          int32_t* iters, double* relres, tp_solve_summary* summary, hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    SolveWork w{};
    tp_status st = static_solve_work(&w);
    if (st != TP_OK) return st;
    const int64_t need = solve_parts_bound(*plan);
    if (need > w.cap)
        return set_error(TP_ERR_ARG, "tp_solve_static: the solve of this plan may need " + std::to_string(need) +
                                         " per-workgroup partial summaries, more than the static workspace holds (" +
                                         std::to_string(w.cap) + "); use tp_solve");
    return solve_impl(plan, b, x, inner, rtol, maxit, iters, relres, summary, stream, w);
}

tp_status tp_solve_summary_fetch(tp_plan* plan, tp_solve_summary* summary, hipStream_t stream) {
    if (!plan || !summary) return set_error(TP_ERR_ARG, "plan and summary must be non-null");
    SolveSummary hs;
    hipError_t e = hipMemcpyAsync(&hs, plan->summary_dev, sizeof(hs), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_error(e, "solve summary readback");
    summary->max_iters = hs.max_iters;
    summary->n_failed = hs.n_failed;
    double mr;
    std::memcpy(&mr, &hs.max_relres_bits, sizeof(mr));
    summary->max_relres = mr;
    if (hs.nonfinite > 0)
        return set_error(TP_ERR_NONFINITE, std::to_string(hs.nonfinite) + " blocks had a non-finite residual");
    if (hs.n_failed > 0) return set_error(TP_ERR_NOT_CONVERGED, std::to_string(hs.n_failed) + " blocks missed rtol");
    return TP_OK;
}

tp_status tp_graph_create(tp_plan* plan, tp_graph_op what, tp_operator op, tp_dtype dtype, const void* in,
                          void* out, double rtol, int32_t maxit, int32_t* iters, double* relres, tp_graph** graph) {
    if (!plan || !graph) return set_error(TP_ERR_ARG, "plan and graph must be non-null");
    *graph = nullptr;
    if (hermite_wave(*plan)) return hermite_wave_error();
    if (what < TP_GRAPH_APPLY || what > TP_GRAPH_SOLVE) return set_error(TP_ERR_ARG, "invalid graph op");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_error(e, "capture stream");
    // one untimed call first so that per-kernel launch parameters are cached
    // outside the capture
    tp_status st = TP_OK;
    auto record = [&](hipStream_t s) -> tp_status {
        switch (what) {
            case TP_GRAPH_APPLY: return tp_apply(plan, op, in, out, dtype, s);
            case TP_GRAPH_INVERSE: return tp_apply_inverse(plan, in, out, dtype, s);
            case TP_GRAPH_SOLVE:
                return tp_solve(plan, static_cast<const double*>(in), static_cast<double*>(out), dtype, rtol, maxit,
                                iters, relres, nullptr, s);
        }
        return set_error(TP_ERR_ARG, "invalid graph op");
    };
    st = record(cs);
    if (st == TP_OK) {
        e = hipStreamSynchronize(cs);
        if (e != hipSuccess) st = hip_error(e, "warm-up call");
    }
    tp_graph* g = nullptr;
    if (st == TP_OK) {
        g = new (std::nothrow) tp_graph();
        if (!g) st = set_error(TP_ERR_OOM, "host allocation failed");
    }
    if (st == TP_OK) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) st = hip_error(e, "hipStreamBeginCapture");
    }
    if (st == TP_OK) {
        tp_status rs = record(cs);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cs, &gr);
        if (rs != TP_OK) st = rs;
        else if (e != hipSuccess) st = hip_error(e, "hipStreamEndCapture");
        g->graph = gr;
        if (st != TP_OK && gr) (void)hipGraphDestroy(gr), g->graph = nullptr;
    }
    if (st == TP_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_error(e, "hipGraphInstantiate");
    }
    (void)hipStreamDestroy(cs);
    if (st != TP_OK) {
        if (g) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            delete g;
        }
        return st;
    }
    *graph = g;
    return TP_OK;
}

tp_status tp_graph_launch(tp_graph* graph, hipStream_t stream) {
    if (!graph || !graph->exec) return set_error(TP_ERR_ARG, "graph is null");
    hipError_t e = hipGraphLaunch(graph->exec, stream);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    return TP_OK;
}

tp_status tp_graph_destroy(tp_graph* graph) {
    if (!graph) return TP_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return TP_OK;
}

tp_status tp_pack(tp_plan* plan, const void* canonical, void* blocked, tp_dtype dtype, hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!valid_dtype(dtype)) return set_error(TP_ERR_UNSUPPORTED, "invalid dtype");
    if (plan->vec_elems > 0 && (!canonical || !blocked)) return set_error(TP_ERR_ARG, "null buffer");
    for (const auto& g : plan->groups) {
        tp_status st = launch_pack(g, canonical, blocked, esize_of(dtype), true, stream);
        if (st != TP_OK) return st;
    }
    return TP_OK;
}

tp_status tp_unpack(tp_plan* plan, const void* blocked, void* canonical, tp_dtype dtype, hipStream_t stream) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!valid_dtype(dtype)) return set_error(TP_ERR_UNSUPPORTED, "invalid dtype");
    if (plan->vec_elems > 0 && (!canonical || !blocked)) return set_error(TP_ERR_ARG, "null buffer");
    for (const auto& g : plan->groups) {
        tp_status st = launch_pack(g, blocked, canonical, esize_of(dtype), false, stream);
        if (st != TP_OK) return st;
    }
    return TP_OK;
}

tp_status tp_plan_autotune(tp_plan* plan, tp_dtype dtype, int32_t reps, double* us) {
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!valid_dtype(dtype)) return set_error(TP_ERR_UNSUPPORTED, "invalid dtype");
    if (plan->persistent) return autotune_persistent(plan, dtype, reps, us);
    if (plan->basis == TP_BASIS_HERMITE)
        return set_error(TP_ERR_UNSUPPORTED, "plans in the Hermite-type basis run the lane kernels only");
    if (reps <= 0) reps = 10;
    const size_t ng = plan->groups.size();
    if (us)
        for (size_t i = 0; i < 3 * ng; ++i) us[i] = -1.0;
    if (plan->vec_elems == 0) return TP_OK;
    const bool inv = plan->inverse_op >= 0 && plan->factor_mode == TP_FACTOR_SCALED;
    const bool solve = inv && plan->inverse_op == TP_OP_CELL;
    TuneBench tb;
    tp_status st = tb.init(plan, dtype, solve, reps);
    for (size_t gi = 0; st == TP_OK && gi < ng; ++gi) {
        GroupInfo& g = plan->groups[gi];
        if (g.nblocks == 0 || g.factors) continue;
        struct Cand { int kind, div; };
        std::vector<Cand> cands;
        if (g.n <= kLaneMaxN) cands.push_back({KIND_LANE, 1});
        cands.push_back({KIND_WAVE, 1});
        cands.push_back({KIND_WAVE, 2});
        cands.push_back({KIND_WAVE, 0});
        if (mfma_eligible(g, dtype, tb.U[0], tb.V[0])) cands.push_back({KIND_MFMA, 1});
        for (int call = 0; st == TP_OK && call < (inv ? 2 : 1); ++call) {
            int8_t* tk = call == 0 ? &g.tune_apply[dtype] : &g.tune_inverse[dtype];
            int8_t* td = call == 0 ? &g.div_apply[dtype] : &g.div_inverse[dtype];
            double best = 1e300;
            Cand bc = cands[0];
            for (const Cand& c : cands) {
                *tk = static_cast<int8_t>(c.kind);
                *td = static_cast<int8_t>(c.div);
                double t = 0.0;
                st = tb.time(
                    [&] {
                        tb.cur = (tb.cur + 1) % tb.nsets;
                        return call == 0 ? group_apply(*plan, g, TP_OP_NEUMANN, tb.U[tb.cur], tb.V[tb.cur], dtype, tb.s)
                                         : group_inverse(*plan, g, tb.U[tb.cur], tb.V[tb.cur], dtype, tb.s);
                    },
                    &t);
                if (st != TP_OK) break;
                if (t < best) best = t, bc = c;
            }
            *tk = static_cast<int8_t>(bc.kind);
            *td = static_cast<int8_t>(bc.div);
            if (us && st == TP_OK) us[3 * gi + call] = best;
        }
        if (st == TP_OK && solve && g.n <= kLaneMaxN) {
            double best = 1e300;
            int8_t bk = KIND_WAVE;
            for (int8_t k : {static_cast<int8_t>(KIND_LANE), static_cast<int8_t>(KIND_WAVE)}) {
                g.tune_solve = k;
                double t = 0.0;
                st = tb.time(
                    [&] {
                        int64_t np = 0;
                        tp_status r = launch_fill(tb.x, plan->vec_elems, TP_F64, 0, true, tb.s);
                        if (r != TP_OK) return r;
                        return group_solve(*plan, g, static_cast<const double*>(tb.b), static_cast<double*>(tb.x),
                                           TP_F64, 1e-10, 20, nullptr, nullptr, plan_work(*plan), 0, &np, tb.s);
                    },
                    &t);
                if (st != TP_OK) break;
                if (t < best) best = t, bk = k;
            }
            g.tune_solve = bk;
            if (us && st == TP_OK) us[3 * gi + 2] = best;
        }
    }
    return st;
}

int32_t tp_plan_group_kernel(const tp_plan* plan, int32_t group, int32_t call, tp_dtype dtype) {
    if (!plan || group < 0 || group >= static_cast<int32_t>(plan->groups.size()) || !valid_dtype(dtype)) return -1;
    const GroupInfo& g = plan->groups[group];
    if (plan->persistent) {
        if (call < 0 || call > 2) return -1;
        const PersistCfg& c = plan->pcfg[call][dtype];
        int pos = 0;
        while (pos < static_cast<int>(c.order.size()) && c.order[pos] != group) ++pos;
        int ltpw = 0;
        while ((1 << ltpw) < c.tpw[group]) ++ltpw;
        const int kind = (call != PCALL_SOLVE && c.lane[group] && persistent_lane_ok(*plan, g)) ? KIND_LANE : KIND_WAVE;
        return kind | (call == PCALL_SOLVE ? c.grid << 4 : 0) | (ltpw << 8) | (pos << 12);
    }
    // alignment-independent view: MFMA eligibility assumes 16-byte aligned vectors
    alignas(16) static const double probe[2] = {0.0, 0.0};
    const void* a = probe;
    switch (call) {
        case 0: {
            const int k = apply_kind(*plan, g, dtype, a, a);
            return k == KIND_WAVE ? k | (g.div_apply[dtype] << 4) : k;
        }
        case 1: {
            const int k = inverse_kind(*plan, g, dtype, a, a);
            return k == KIND_WAVE ? k | (g.div_inverse[dtype] << 4) : k;
        }
        case 2: return solve_kind(*plan, g);
    }
    return -1;
}

}  // extern "C"
