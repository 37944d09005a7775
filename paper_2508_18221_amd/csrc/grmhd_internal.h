// Internal declarations of the gfx950 BSSN + Valencia GRMHD spectral stage.
// Layout of the device buffers and the launch interface between the host
// orchestration (abi.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "grmhd.h"

namespace grmhd {

constexpr int NF = 32;    // evolved fields
constexpr int NFA = 33;   // fields per stored state: the 32, then psi (GLM contexts)
constexpr int ND1 = 21;   // fields with first derivatives (0..20)
constexpr int ND2 = 11;   // fields with second derivatives
// fields with second derivatives: phi, gt_ij, alpha, beta^i
constexpr int D2_FIELD[ND2] = {0, 1, 2, 3, 4, 5, 6, 17, 18, 19, 20};
// fields with first derivatives only: At_ij, K, Gt^i
constexpr int D1_ONLY[10] = {7, 8, 9, 10, 11, 12, 13, 14, 15, 16};

// Scratch buffer: fields of P doubles.
enum : int {
  SC_US = 0,      // 33  stage state U^(s) (+ psi)
  SC_ACC = 33,    // 33  RK accumulator (+ psi)
  SC_FLUX = 66,   // 24  alpha sqrt(gamma) F^a of var v at SC_FLUX + 8a + v
  SC_D1 = 90,     // 63  d_a f at SC_D1 + 21a + f (f = 0..20)
  SC_D2 = 153,    // 33  d_a d_a of second-derivative field s at SC_D2 + 11a + s
  SC_MX = 186,    // 33  mixed (r th, r ph, th ph) at SC_MX + 11m + s
  SC_DF = 219,    // 24  d_a (alpha sqrt(gamma) F^a_v) at SC_DF + 8a + v
  SC_GLM = 243,   // 6   GLM: d_a (sqrt(gamma) B^a) at SC_GLM + a, d_a psi at SC_GLM + 3 + a
                  // 249..254 unused
  SC_BG = 255,    // 33  fixed-background form: d_a of background field s at SC_BG + 11a + s
                  //     (s: phi, gt_ij, alpha, beta^i, the D2_FIELD order);
                  //     coupled RK4 step: the second stage state (SC_US2_COUPLED)
  SC_NFIELDS = 288
};
// The RK4 stages alternate between two stage states: SC_US and this block
// (coupled form: SC_BG, free there; fixed-background form and the split
// step's fluid stages: SC_D2, which they leave unused).
constexpr int SC_US2_COUPLED = SC_BG;
constexpr int SC_US2_FIXED = SC_D2;

// Resident buffer: fields of P doubles, then operators and small arrays.
enum : int {
  RS_U = 0,       // 33  state U^n (+ psi)
  RS_K0 = 33,     // 1   static 1+log source
  RS_PRIM = 34,   // 5   rho, p, v^r, v^th, v^ph (last recovery; warm start)
  RS_FAIL = 39,   // 1   1.0 where the atmosphere policy was taken
  RS_NFIELDS = 40
};

// Operators per axis: first derivative, second derivative, filter.
enum : int { OP_D1 = 0, OP_D2 = 1, OP_FILT = 2 };

inline int round_up(int n, int m) { return (n + m - 1) / m * m; }

// One contraction task: out_m = A_m applied along the axis to `src`.
struct Task {
  int src_sel, src;     // base selector, field index
  int src_f32;          // 1: the input field is FP32 (FP32 outputs only)
  int dst_sel, dst0;    // destination of matrix 0
  int dst1;             // destination of matrix 1 (same base as dst0)
  int nmat;             // operators this task applies (1 or 2)
  int op;               // nmat == 1: which operator (0 or 1; copy-ahead kernels of the strided axes)
};
constexpr int MAX_TASKS = 64;
struct TaskList {
  int n;
  Task t[MAX_TASKS];
};
// Up to four base pointers a task can address (selectors 0..3).
struct Bases {
  double* b[4];
};

// Reduced-precision contraction task: input may be FP64 or FP32, output FP32.
struct MixedTask {
  int src_sel, src, src_f32;
  int dst_sel, dst0, dst1;
  int nmat;             // operators this task applies (1 or 2)
};
struct MixedTaskList {
  int n;
  MixedTask t[MAX_TASKS];
};
// One operator in the reduced-precision forms: FP32 transposed AT[k][i]
// (padded like the FP64 one) and BF16 high/low parts of A[i][k], row-major,
// i padded to 16 and k padded to 32.
struct MixedOps {
  const float* f32;
  const __bf16* bhi;
  const __bf16* blo;
};

// Jobs advanced by one launch (same grid class, same buffer layout): byte
// offset of job j's buffers from job 0's (its resident and scratch blocks
// move together) and its time step.  A single context is n = 1, d = 0.
constexpr int MAXB = 32;
struct JobSet {
  int n;
  long long d[MAXB];
  double dt[MAXB];
};

template <class T>
__host__ __device__ inline T* shift_ptr(T* p, long long d) {
  return (T*)((char*)p + d);
}

struct PointParams {
  int nr, nth, nph;
  long long P;
  double gamma_ad, eta;
  double gfac, gm1g;  // Gamma/(Gamma-1), (Gamma-1)/Gamma
  int cowling, gauge_k0;
  double rho_floor, p_floor;
  int glm;            // GLM constraint damping on (psi is field 32)
  double ch2, itau;   // c_h^2, 1/tau of the GLM terms
  int c2p_damped;     // primitive recovery by the paper's damped iteration
};

// A folded operator on the device (even N): E^T then O^T, each Hpad x Hpad,
// its centro-symmetry sign, and an optional per-row scale (null: 1).
struct FoldOp {
  const double* et;
  const double* g;
  double sigma;
};

// FP32 folded operator (mixed-precision form): E^T then O^T in FP32, row
// scale in FP64 (null: 1), sign.
struct FoldOp32 {
  const float* et;
  const double* g;
  double sigma;
};

// Host-side operator set (built in long double, stored as double).
struct Operators {
  int n[3];            // nr, nth, nph
  int npad[3];         // padded to multiples of 16
  // transposed, zero-padded: AT[k * npad + i] = A[i][k]
  std::vector<double> at[3][3];   // [axis][op]
  std::vector<double> r, th, ph;  // nodes
  std::vector<double> wr, wth;    // quadrature weights (d r, d theta)
  // reduced-precision copies of the derivative operators (D1, D2 per axis)
  std::vector<float> at32[3][2];
  std::vector<uint16_t> bhi[3][2], blo[3][2];  // bf16 bit patterns, [npad][kpad]
  int kpad[3];
  // even/odd folded forms (even N): unmapped operators, E^T then O^T, [axis][op]
  bool fold[3];
  int hpad[3];                       // round_up(N/2, 16)
  std::vector<double> fmat[3][3];
  std::vector<float> fmat32[3][2];   // FP32 copies of the folded D1, D2
  std::vector<double> gr;            // radial row scales g1, g2, g21 (nr each)
  double Lc, Lh, Tc, Th;
  double dt;
};

void build_operators(const grmhd_grid& g, double cfl, Operators* ops);

// Chebyshev first- and second-derivative matrices on n CGL nodes in the
// reference coordinate (row-major, built in long double and rounded once;
// D2 = D1 D1 with zero row sums), the ones build_operators maps.
void cheb_reference_matrices(int n, std::vector<double>* D1, std::vector<double>* D2);

// Two contexts can share one launch sequence (grmhd_step_batch, the job
// server's classes) when their buffers are laid out alike and the kernels get
// the same parameters and take the same path: same grid sizes, filter and
// dealiasing switches, precision, Gamma, eta, floors and form switches
// (fixed background, 1+log source, GLM with its c_h and tau, split step,
// damped recovery).  Operators, floors and dt are per job.
bool same_step_class(const grmhd_grid& ga, const grmhd_phys& pa, grmhd_prec qa, const grmhd_grid& gb,
                     const grmhd_phys& pb, grmhd_prec qb);

// Parameter checks of grmhd_create; with need_initial_data also the
// conditions under which grmhd_init_state can build its data (black hole,
// perturbation amplitude, field strength, a transonic Michel flow), so that a
// job can be refused when it is submitted.  GRMHD_OK or GRMHD_E_ARG with *err
// set.
int validate_phys(const grmhd_phys& ph, bool need_initial_data, std::string* err);

// Release a context whose work on its stream is known to be complete (its
// last launch sequence's event has been observed), without waiting for that
// stream: other contexts may have work queued there.
void destroy_idle_context(grmhd_ctx* c);

// grmhd_create with the operators of this grid and cfl built beforehand
// (prebuilt: copied into the context; null: built here).  The job server keeps
// one set per grid, so admission does not rebuild them.
int create_context(const grmhd_grid* grid, const grmhd_phys* phys, grmhd_prec prec, void* dev_resident,
                   void* dev_scratch, void* hip_stream, const Operators* prebuilt, grmhd_ctx** out);

// Initial data on the (theta, r) plane (the data are axisymmetric up to the
// seeded perturbation): PL_NFIELDS fields of nr * nth doubles, index k nr + j.
enum : int {
  PL_PHI = 0, PL_GT = 1, PL_AT = 7, PL_K = 13, PL_GAMT = 14, PL_ALPHA = 17, PL_BETAR = 18, PL_K0 = 19,
  PL_RHO = 20, PL_P = 21, PL_V = 22, PL_SB = 25, PL_SQRTG = 28, PL_GM = 29,  // gm: physical metric, 9
  PL_NFIELDS = 38
};
int host_initial_plane(const grmhd_grid& g, const grmhd_phys& ph, const Operators& ops,
                       std::vector<double>* plane, std::string* err);
// The 3D state (fields 0..31) and K0 from the plane fields (device copy):
// spacetime copied along phi; rho (Michel) or p (torus) times
// 1 + amp (2u - 1), u the top 53 bits of SplitMix64(seed ^ n) / 2^53 at point
// n; then the densitised conserved variables.
hipError_t launch_init_expand(const double* plane, int torus, uint64_t seed, double amp, double gamma_ad,
                              const PointParams& pp, double* U, double* K0, hipStream_t s);

// ---- conformally flat initial data (xcts.hip) ----------------------------
struct XctsGrid {
  int nr, nth, nph;
  double Lh, Th;        // radial log-map and polar affine-map half widths
  const double* r;      // radial nodes (host, nr)
  const double* th;     // polar nodes (host, nth)
};
// Doubles of host-built operators the solver stages after its five work
// arrays of P doubles in the work buffer.
size_t xcts_operator_doubles(int nr, int nth, int nph);
// Picard iteration for Lap psi = -2 pi E psi^5 on the grid, the boundary
// values of psi (device, P doubles; in: the initial guess carrying the
// Dirichlet data, out: the solution) held; E device, P doubles.  work: at
// least 5 P + xcts_operator_doubles(...) doubles of device memory; partials:
// device memory for 2 x partial_blocks doubles.  Syncs s.
int xcts_solve(const XctsGrid& g, double* work, double* partials, int partial_blocks, hipStream_t s,
               const double* E, double* psi, int max_iter, double tol, int* iters, double* change,
               std::string* err);

// ---- kernel launchers (kernels.hip) --------------------------------------
// Contraction along axis (0 r, 1 theta, 2 phi) with nmat = 1 or 2 matrices.
// Storage of a contraction's input and output fields (the arithmetic is
// FP64): both FP64; FP64 in, FP32 out; both FP32 (field g of an FP32 block at
// float offset g P from the base pointer).
enum { IO_F64 = 0, IO_OUT_F32 = 1, IO_F32 = 3 };
hipError_t launch_contract(int axis, int nmat, const TaskList& tl, const Bases& B,
                           const double* AT0, const double* AT1, const int n[3],
                           const int npad[3], long long P, const JobSet& js, hipStream_t s,
                           int io = IO_F64);
hipError_t launch_contract_mixed(int prec, int axis, int nmat, const MixedTaskList& tl, const Bases& B,
                                 const MixedOps& op0, const MixedOps& op1, const int n[3],
                                 const int npad[3], long long P, const JobSet& js, hipStream_t s);
hipError_t set_mixed_kernel_attributes();
// Folded contraction (even N): out_0 = g0 . (A_0 u), out_1 = g1 . (A_1 u) + g10 . (A_0 u);
// nmat = 2 lets each task apply one or two operators (its own nmat)
hipError_t launch_contract_fold(int axis, int nmat, const TaskList& tl, const Bases& B, const FoldOp& op0,
                                const FoldOp& op1, const double* g10, const int n[3], const int hpad[3],
                                long long P, const JobSet& js, hipStream_t s, int io = IO_F64);
hipError_t set_fold_kernel_attributes();
hipError_t launch_contract_f32_fold(int axis, int nmat, const MixedTaskList& tl, const Bases& B,
                                    const FoldOp32& op0, const FoldOp32& op1, const double* g10, const int n[3],
                                    const int hpad[3], long long P, const JobSet& js, hipStream_t s);
// floors: rho floor at the nr radial nodes, then the p floor; the metric
// (phi, gt_ij, alpha, beta^i) is read from Ug, the GRMHD fields from U
hipError_t launch_c2p_flux(const double* U, const double* Ug, double* prim, double* fail, double* flux,
                           const double* floors, const PointParams& pp, const JobSet& js, hipStream_t s);
// mode 0: out = L(U_s); 1..4: classic RK4 stage s; 5: forward Euler of the
// spacetime fields (split step; Us = Un = out).  der: derivative arrays
// (scratch fields SC_D1 .. SC_DF + 23, in that order), FP64 or FP32.  In
// modes 0..4 out shares no location with Us, Un or acc (stage 4 may write
// the Un buffer: it does not read Un), and acc none with Us or Un.  Mode 1
// takes Us as U^n (Un is not read).
hipError_t launch_rhs_rk(int mode, bool der_f32, const double* Us, const void* der, const double* prim,
                         const double* K0, const double* Un, double* acc, double* out, const PointParams& pp,
                         const JobSet& js, hipStream_t s);
// Fixed-background form: GRMHD (and psi) right-hand sides / RK4 stage from the
// stage fluid Us, background state Ug, background first derivatives bg
// (SC_BG block) and the flux derivative arrays (der as in launch_rhs_rk; the
// same rules for the buffers and for mode 1).
hipError_t launch_rhs_fixed(int mode, bool der_f32, const double* Us, const double* Ug, const double* bg,
                            const void* der, const double* prim, const double* Un, double* acc, double* out,
                            const PointParams& pp, const JobSet& js, hipStream_t s);
// Hamiltonian constraint H and momentum-constraint norm |M| (P doubles each)
// from FP64 derivative arrays
hipError_t launch_ham(const double* U, const double* der, double* H, double* Mn, const PointParams& pp,
                      hipStream_t s);
hipError_t launch_k0(const double* U, const double* scr, double* K0, const PointParams& pp,
                     hipStream_t s);
// Per-block partial reductions for diagnostics: writes nblocks x DIAG_Q doubles.
// [0] rest mass, [1] entropy, [2] fails, [3] non-finite, [4] max|div B|,
// [5] min alpha, [6] max W, [7] sum H^2 w, [8] max|H|, [9] sum w,
// [10] sum |M|^2 w, [11] max |M|
constexpr int DIAG_Q = 12;
hipError_t launch_diag_partials(const double* U, const double* prim, const double* fail,
                                const double* scr, const double* H, const double* Mn, const double* wr,
                                const double* wth, double gamma_ad, const PointParams& pp,
                                double* partials, int* nblocks, hipStream_t s);
int diag_partials_blocks(long long P);
hipError_t set_kernel_attributes();

// ---- helpers of the copy-ahead contraction pipelines ---------------------------
// s_waitcnt immediate: vector-memory count n (0..63), no wait on the others
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }

typedef __attribute__((address_space(3))) void lds_void_t;

// Workgroup barrier for the copy pipelines: LDS reads done, then s_barrier.
// The copies a barrier needs are waited for explicitly before it (the
// compiler may otherwise wait for every outstanding copy and store there).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

}  // namespace grmhd
