// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/tpfdm.h"

namespace tpfdm {

constexpr int kMinN = 2;
constexpr int kMaxN = 8;
// degrees n <= kLaneMaxN run one block per lane; larger n one block per wave
constexpr int kLaneMaxN = 4;  // apply / apply_inverse only

// ---------------------------------------------------------------- refdata
void gll_points(int n, double* x);
void gauss_points(int nq, double* x, double* w);
void reference_matrices(int n, double C, double* M, double* K, double* A);
int gen_eigen(int n, const double* M, const double* P, double* S, double* lam);
void endpoint_derivatives(int n, double* g0, double* g1);
void prolongation_1d(int n, double* P0, double* P1);
// Hermite-type basis: T[i * n + j] = psi_j(x_i) at the Gauss-Lobatto nodes (n >= 4).
// hermite_sign(n, i): -1 for the derivative-at-1 function (i = n - 2), else 1;
// conjugated by this sign the basis is symmetric under x -> 1 - x.
__host__ __device__ constexpr double hermite_sign(int n, int i) { return i == n - 2 ? -1.0 : 1.0; }
void hermite_transform(int n, double* T);
bool invert_small(int n, const double* A, double* Ai);
// X <- T^T X T.
void congruence(int n, const double* T, double* X);
// Reference 1D factors of a vertex patch of two cells of nc points each
// (n = 2 nc): blockdiag mass and stiffness, and the patch operator.
void patch_reference(int nc, double C, double* M, double* K, double* A);

// Even-odd tables of the centrosymmetric 1D factors, one slot of kEOSlot
// elements per (n, table, element type):
//   EO_APPLY_K / EO_APPLY_A:  ME[hc][hc] | MO[h][h] | PE[hc][hc] | PO[h][h]
//   EO_INV:                   SE[hc][hc] | SO[h][h] | lam[n] (split order)
// with h = n/2, hc = (n+1)/2.  Element type 0 = double, 1 = float.
//   EO_PLAIN_K / EO_PLAIN_A:  M[n][n] | P[n][n]   (plain, for the lane kernels)
//   EO_PLAIN_S:               S[n][n] | lam[n]
//   EO_APPLY_F:               ME | MO | FE | FO with F = A_hat - K_hat (the
//                             face part of a mesh cell's diagonal block)
enum {
    EO_APPLY_K = 0, EO_APPLY_A = 1, EO_INV = 2, EO_PLAIN_K = 3, EO_PLAIN_A = 4, EO_PLAIN_S = 5, EO_APPLY_F = 6,
    EO_NTAB = 7
};
constexpr int kEOSlot = 64;
// Builds ME|MO|PE|PO from centrosymmetric M and P; false when either is not.
bool build_eo_apply(int n, const double* M, const double* P, double* out);
// Builds SE|SO|lam from eigenvectors S (columns) and eigenvalues; makes every
// column exactly symmetric or antisymmetric.  False when the parity split
// does not have ceil(n/2) symmetric columns.
bool build_eo_inverse(int n, const double* S, const double* lam, double* out);

// ---------------------------------------------------------------- plan data
struct RefData {
    bool built = false;
    double M[kMaxN * kMaxN];
    double K[kMaxN * kMaxN];
    double A[kMaxN * kMaxN];
    double g0[kMaxN], g1[kMaxN];           // endpoint derivatives of the basis
    double P0[kMaxN * kMaxN], P1[kMaxN * kMaxN];   // embeddings into the two children
    double T[kMaxN * kMaxN], Ti[kMaxN * kMaxN];    // nodal <- basis coefficients, and back
    // fast-diagonalization factors of the operator chosen at setup
    bool eig_ready = false;
    double S[kMaxN * kMaxN];
    double lam[kMaxN];
};

struct GroupInfo {
    int n;
    int logB;
    int64_t nblocks;
    int64_t offset;       // element offset of the group in blocked vectors
    int64_t canon;        // element offset in canonical order
    int64_t block0;       // first global block index of the group
    double* h;            // plan-owned device copy, [nblocks][3]
    bool lane_solve;      // solve with one block per lane (else one wave per tile)
    // GENERAL mode (plan-owned device memory, null when unused)
    bool factors = false;     // the group is given by per-block factors (no h)
    double* fac = nullptr;    // [nblocks][3][2][n][n] (M_d, P_d) FP64
    float* fac32 = nullptr;   // same in FP32
    double* eig = nullptr;    // [nblocks][3][n*n + n] (S_d, lam_d) FP64
    float* eig32 = nullptr;   // same in FP32
    // choices of tp_plan_autotune (-1: the default rule), per storage dtype
    int8_t tune_apply[4] = {-1, -1, -1, -1};    // KIND_LANE / KIND_WAVE / KIND_MFMA
    int8_t tune_inverse[4] = {-1, -1, -1, -1};
    int8_t tune_solve = -1;                      // KIND_LANE / KIND_WAVE
    // wave kernels: persistent grid divisor (0: one workgroup per tile); the
    // default is the occupancy grid for FP64 and one workgroup per tile for
    // the 2- and 4-byte types (measured faster at n = 8)
    int8_t div_apply[4] = {1, 0, 0, 0};
    int8_t div_inverse[4] = {1, 0, 0, 0};
};

// Kernel families of a group's call (tp_plan_group_kernel reports these).
enum { KIND_LANE = 0, KIND_WAVE = 1, KIND_MFMA = 2, KIND_GENERAL = 3 };

// Single-launch configuration of a persistent plan for one call (apply,
// apply_inverse, solve) and dtype: per group the tile body (one block per
// lane for n <= 4, or one wave per tile) and the tiles each workgroup runs,
// the order of the groups' segments in the launch, and for the solve the
// grid.  Defaults follow the plan's mapping; tp_plan_autotune replaces them
// with measured choices.
struct PersistCfg {
    std::vector<int8_t> lane;     // per group: 1 = lane-per-block body
    std::vector<int8_t> tpw;      // per group: consecutive tiles per workgroup (1, 2, 4, 8)
    std::vector<int32_t> order;   // group index of each segment, in launch order
    int8_t grid = 1;              // solve: 1 occupancy grid, 2 half of it, 0 one workgroup per item
    int64_t items = 0;            // work items of the launch (set when uploaded)
    bool tuned = false;
};
enum { PCALL_APPLY = 0, PCALL_INVERSE = 1, PCALL_SOLVE = 2 };

struct Plan {
    int device = 0;
    double penalty_C = 2.0;
    bool persistent = false;
    int mapping = 0;
    std::vector<GroupInfo> groups;
    RefData ref[kMaxN + 1];
    int inverse_op = -1;
    int factor_mode = 0;           // tp_factor_mode of the last successful setup
    int64_t vec_elems = 0;
    int64_t ndof = 0;
    int64_t nblocks = 0;
    // device workspace
    void* summary_dev = nullptr;   // solve summary of the last solve
    void* summary_host = nullptr;  // pinned, host-coherent copy of it (tp_solve's readback)
    void* summary_host_dev = nullptr;  // the same memory's device address
    int summary_seq = 0;           // tag of the last summary written there
    void* partials_dev = nullptr;  // SolvePartial per workgroup of the last solve
    int64_t partials_cap = 0;
    // MFMA operand tables for n = 8 FP16 / BF16: apply [K or A][f16 or bf16], inverse [f16 or bf16]
    void* mfma_apply_dev[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void* mfma_inv_dev[2] = {nullptr, nullptr};
    void* segs_dev = nullptr;      // persistent-kernel segment tables: one per (call, dtype), ngroups each
    PersistCfg pcfg[3][4];         // their configurations [PCALL_*][tp_dtype]
    void* eo_dev = nullptr;        // even-odd tables, (kMaxN+1) x EO_NTAB x 2 slots
    int64_t wave_grid = 2048;      // persistent grid of the wave kernels
    int cus = 256;                 // compute units of the plan's device
    // uniform box mesh of tp_plan_create_mesh (one group, cells in mesh order)
    int basis = 0;                 // tp_basis of every block's coefficients
    bool patches = false;          // blocks are vertex patches (reference tables of two cells)
    bool mesh = false;
    int mesh_m[3] = {0, 0, 0};
    double mesh_h[3] = {0.0, 0.0, 0.0};
};

// Per-workgroup partial summary of a solve launch (plain stores, no atomics).
struct SolvePartial {
    int max_iters;
    int n_failed;
    int nonfinite;
    int pad;
    double max_relres;
};
// Maximum one-wave workgroups resident per CU (sizes the partials array).
constexpr int kMaxWgPerCu = 32;

// Device-side solve summary, written by the reduction kernel after a solve.
struct SolveSummary {
    int max_iters;
    int n_failed;
    int nonfinite;
    int pad;
    unsigned long long max_relres_bits;
};

// Where a solve launch writes its per-workgroup partial summaries (at most
// cap of them) and where the reduction puts the summary: the plan's own
// workspace for tp_solve, the library's static scratch for tp_solve_static.
struct SolveWork {
    SolvePartial* parts;
    int64_t cap;
    SolveSummary* summary;
    SolveSummary* host = nullptr;   // device address of pinned host memory for the readback, or null
};
inline SolveWork plan_work(const Plan& p) {
    return SolveWork{static_cast<SolvePartial*>(p.partials_dev), p.partials_cap,
                     static_cast<SolveSummary*>(p.summary_dev), static_cast<SolveSummary*>(p.summary_host_dev)};
}

// The static device workspace of tp_solve_static (static_scratch.hip): its
// address on the current device, looked up on the first call per device.
tp_status static_solve_work(SolveWork* out);

// thread-local last error
tp_status set_error(tp_status st, const std::string& msg);
tp_status hip_error(int err, const char* what);

// ---------------------------------------------------------------- launchers
// All return TP_OK or TP_ERR_HIP/TP_ERR_UNSUPPORTED.
tp_status launch_apply(const Plan& plan, const GroupInfo& g, const double* Pm, const void* u,
                       void* v, tp_dtype dt, hipStream_t s);
tp_status launch_inverse(const Plan& plan, const GroupInfo& g, const void* r, void* x,
                         tp_dtype dt, hipStream_t s);
// Solve launchers write one SolvePartial per workgroup starting at
// partials + part_base and report the number written in *nparts.
tp_status launch_solve(const Plan& plan, const GroupInfo& g, const double* b, double* x,
                       tp_dtype inner, double rtol, int maxit, int32_t* iters,
                       double* relres, const SolveWork& w, int64_t part_base, int64_t* nparts, hipStream_t s);
// Lane-per-block solve (n <= 4); same contract as launch_solve.
tp_status launch_solve_lane(const Plan& plan, const GroupInfo& g, const double* b, double* x,
                            tp_dtype inner, double rtol, int maxit, int32_t* iters,
                            double* relres, const SolveWork& w, int64_t part_base, int64_t* nparts, hipStream_t s);
// GENERAL mode: per-block factors and eigen-decompositions (general.hip).
tp_status launch_apply_gen(const Plan& plan, const GroupInfo& g, const void* u, void* v, tp_dtype dt,
                           hipStream_t s);
tp_status launch_inverse_gen(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                             hipStream_t s);
tp_status launch_solve_gen(const Plan& plan, const GroupInfo& g, const double* b, double* x, tp_dtype inner,
                           double rtol, int maxit, int32_t* iters, double* relres, const SolveWork& w,
                           int64_t part_base, int64_t* nparts, hipStream_t s);
// Fills n elements of dtype dt with pseudo-random values in [-1, 1]
// (a counter hash of the element index and seed), or zero when zero is set.
tp_status launch_fill(void* dst, int64_t n, tp_dtype dt, uint64_t seed, bool zero, hipStream_t s);
// to_blocked: src canonical -> dst blocked; otherwise src blocked -> dst canonical
tp_status launch_apply_eo(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v,
                          tp_dtype dt, hipStream_t s);
tp_status launch_inverse_eo(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                            hipStream_t s);
inline const void* eo_table(const Plan& plan, int n, int tab, int et) {
    return static_cast<const char*>(plan.eo_dev) +
           static_cast<size_t>(((n * EO_NTAB + tab) * 2 + et) * kEOSlot) * sizeof(double);
}
tp_status upload_eo(Plan& plan, int n, int tab, const double* vals, int count);
// MFMA path (n = 8, FP16 / BF16, B = 1, 16-byte aligned vectors).
bool build_mfma_tables(const double* M, const double* P, const double* S, const double* lam, bool bf16,
                       std::vector<uint16_t>* apply, std::vector<uint8_t>* inverse);
bool mfma_eligible(const GroupInfo& g, tp_dtype dt, const void* a, const void* b);
tp_status launch_apply_mfma(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v, tp_dtype dt,
                            hipStream_t s);
tp_status launch_inverse_mfma(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                              hipStream_t s);

// Persistent single-launch paths over all groups of a plan.
// persistent_setup allocates the segment tables and uploads the default
// configuration of every call and dtype; persistent_upload rewrites the
// table of one (call, dtype) from plan.pcfg (host-synchronous: no launch
// that reads that table may be in flight).
tp_status persistent_setup(Plan& plan);
tp_status persistent_upload(Plan& plan, int call, int dt);
// Whether group g may run the lane-per-block body in a single launch.
bool persistent_lane_ok(const Plan& plan, const GroupInfo& g);
tp_status launch_apply_persistent(const Plan& plan, int op, const void* u, void* v, tp_dtype dt, hipStream_t s);
tp_status launch_inverse_persistent(const Plan& plan, const void* r, void* x, tp_dtype dt, hipStream_t s);
tp_status launch_solve_persistent(const Plan& plan, const double* b, double* x, tp_dtype inner, double rtol,
                                  int maxit, int32_t* iters, double* relres, const SolveWork& w, int64_t* nparts,
                                  hipStream_t s);
// Multigrid V-cycle of a mesh plan (mg.hip): u = V(b) on the finest level,
// every kernel skipped once the PCG state st (nullable) is done; the dot
// kernel writes per-tile partials of (a, b).
tp_status mg_enqueue_vcycle(const tp_mg* m, const double* b, double* u, const void* st, bool f32, hipStream_t s);
// With FP32 level storage the V-cycle's result stays on the device in the
// hierarchy's finest FP32 vector (u may then be null): mg_result32 returns
// it, mg_enqueue_widen copies it to an FP64 vector; null / TP_ERR_STATE for
// FP64 storage.
int mg_storage(const tp_mg* m);
const float* mg_result32(const tp_mg* m);
tp_status mg_enqueue_widen(const tp_mg* m, double* dst, hipStream_t s);
// Partial (a, b) per 64-cell tile with b in FP64 or (b32) FP32.
tp_status mg_enqueue_dot(const tp_mg* m, const double* a, const void* b, bool b32, double* part, const void* st,
                         hipStream_t s);
const tp_plan* mg_plan(const tp_mg* m);
// Coupled SIPG operator of a mesh plan (sipg.hip): A u, or A^face u when face_only.
tp_status launch_sipg(const Plan& plan, const GroupInfo& g, bool face_only, const void* u, void* v, tp_dtype dt,
                      hipStream_t s);
tp_status launch_pack(const GroupInfo& g, const void* src, void* dst, int esize,
                      bool to_blocked, hipStream_t s);
tp_status launch_summary_reduce(const SolveWork& w, int64_t nparts, SolveSummary* host_out, int tag, hipStream_t s);

}  // namespace tpfdm

// The opaque handle of the C ABI is the plan itself.
struct tp_plan : public tpfdm::Plan {};
