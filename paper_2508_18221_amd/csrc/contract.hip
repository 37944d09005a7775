// Dense spectral-operator contractions along grid lines on FP64 MFMA (gfx950).
//
// Every derivative and filter of the method (Methods, "The Spectral Derivative
// Operators", "Dealiasing and Spectral Filtering") is a dense N x N matrix
// applied along one coordinate of fields laid out [phi][theta][r] (r fastest):
//   axis r     : out[line][i]    = sum_k A[i][k] in[line][k]     (lines = th*ph)
//   axis theta : out[o][i][c]    = sum_k A[i][k] in[o][k][c]     (o = phi, c = r)
//   axis phi   : out[i][c]       = sum_k A[i][k] in[k][c]        (c = theta*r)
// A workgroup stages one input tile [k = 0..Npad) x [64 columns] in LDS
// (columns are r-lines for the r axis, contiguous inner points otherwise),
// reads each input element from HBM once, and applies one or two operators
// (first and second derivative share the read).  Operators are read
// transposed (AT[k][i]) from L2 as MFMA fragments.
//
// MFMA v_mfma_f64_16x16x4_f64 fragment layout (wave64):
//   A operand (16x4):  lane l holds A[l % 16][l / 16]
//   B operand (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16, 4 regs): lane l, reg v holds D[(l / 16) + 4 v][l % 16]
// (the f64 accumulator interleaves rows by 4, unlike the f32 16x16x4 form).
#include "grmhd_internal.h"

#include <algorithm>
#include <type_traits>

namespace grmhd {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TILE_COLS = 64;
constexpr int LDS_STRIDE = 72;  // doubles: rows 16 banks apart, so the 4 rows a
                                // fragment read touches hit each bank twice
constexpr int NARROW = 32;     // tile columns on the strided axes at N = 128
constexpr int KC = 4;           // k-steps (of 4) of operator fragments held in registers

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The tasks of tl whose input storage is FP32 (f32 = 1) or FP64 (f32 = 0).
static TaskList tasks_with_input(const TaskList& tl, int f32) {
  TaskList out;
  out.n = 0;
  for (int i = 0; i < tl.n; ++i)
    if ((tl.t[i].src_f32 != 0) == (f32 != 0)) out.t[out.n++] = tl.t[i];
  return out;
}

static bool any_f32_input(const TaskList& tl) {
  for (int i = 0; i < tl.n; ++i)
    if (tl.t[i].src_f32) return true;
  return false;
}

// INNER = true : r axis (tile columns are r-lines, output rows are lines)
// INNER = false: theta / phi axes (tile columns are contiguous inner points)
// IT, OT: storage type of the input and output fields (double, or float for
// the FP32 derivative arrays of the FP32-storage form; the arithmetic is FP64
// either way, a float field of the block sits at float offset field x P).
template <int NMAT, bool INNER, int WI, typename IT = double, typename OT = double>
__global__ __launch_bounds__(256) void k_contract(TaskList tl, Bases B,
                                                  const double* __restrict__ AT0,
                                                  const double* __restrict__ AT1, int N, int Npad,
                                                  int inner, int slab, long long P, JobSet js) {
  extern __shared__ double tile[];  // [Npad][LDS_STRIDE]
  const Task tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];  // this job's buffer offset
  AT0 = shift_ptr(AT0, jd);
  AT1 = shift_ptr(AT1, jd);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c0 = blockIdx.x * TILE_COLS;
  const size_t off = (size_t)blockIdx.y * (size_t)slab;
  const IT* __restrict__ src = (const IT*)shift_ptr(B.b[tk.src_sel], jd) + (size_t)tk.src * (size_t)P + off;
  OT* __restrict__ dst0 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P + off;
  OT* __restrict__ dst1 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P + off;

  // ---- stage the input tile ------------------------------------------------
  // LOADS independent global loads per thread are issued before any of them
  // is written to LDS (memory-level parallelism for the HBM stream)
  constexpr int LOADS = 16;
  if (INNER) {
    // 64 consecutive lines of N doubles: contiguous in memory; stored transposed
    const int ncols = min(TILE_COLS, inner - c0);  // lines in this tile
    const IT* __restrict__ s = src + (size_t)c0 * N;
    const int total = TILE_COLS * N, valid = ncols * N;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double v[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        v[q] = (e < valid) ? (double)s[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) {
          const int line = e / N, k = e - line * N;
          tile[k * LDS_STRIDE + line] = v[q];
        }
      }
    }
    for (int e = threadIdx.x; e < (Npad - N) * TILE_COLS; e += 256)
      tile[(N + e / TILE_COLS) * LDS_STRIDE + (e % TILE_COLS)] = 0.0;
  } else {
    const int total = Npad * TILE_COLS;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double v[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        const int k = e >> 6, c = e & 63;
        v[q] = (e < total && k < N && c0 + c < inner) ? (double)src[(size_t)k * inner + c0 + c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) tile[(e >> 6) * LDS_STRIDE + (e & 63)] = v[q];
      }
    }
  }
  __syncthreads();

  // ---- work split: i-tiles (operator rows) x column fragments ---------------
  // WI waves along the operator rows, 4 / WI along the 64 tile columns; each
  // wave owns FW = WI fragments of 16 columns.  Everything inside the k loop
  // is compile-time shaped, so the MFMAs issue back to back on independent
  // accumulators instead of one at a time behind branches.
  constexpr int FW = WI;
  const int T = Npad >> 4;
  const int wi = wave % WI, wf = wave / WI;
  const int lr = lane & 15, lk = lane >> 4;

  const int nks = Npad >> 2;  // k-steps of 4; a multiple of KC since Npad % 16 == 0
  for (int it = wi; it < T; it += WI) {
    d4 acc[NMAT][FW];
#pragma unroll
    for (int m = 0; m < NMAT; ++m)
#pragma unroll
      for (int f = 0; f < FW; ++f) acc[m][f] = d4{0.0, 0.0, 0.0, 0.0};
    const double* __restrict__ a0p = AT0 + (size_t)lk * Npad + it * 16 + lr;
    const double* __restrict__ a1p = (NMAT > 1 ? AT1 : AT0) + (size_t)lk * Npad + it * 16 + lr;
    const double* tp = tile + lk * LDS_STRIDE + wf * FW * 16 + lr;
    // operator fragments of one chunk (KC k-steps) live in registers; the next
    // chunk is requested before the current one is consumed
    double a[NMAT][KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      a[0][q] = a0p[(size_t)(4 * q) * Npad];
      if (NMAT > 1) a[NMAT - 1][q] = a1p[(size_t)(4 * q) * Npad];
    }
    for (int kc = 0; kc < nks; kc += KC) {
      // the last chunk re-requests itself: an in-bounds dummy prefetch
      const int kn = (kc + KC < nks) ? kc + KC : kc;
      double an[NMAT][KC];
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        an[0][q] = a0p[(size_t)(4 * (kn + q)) * Npad];
        if (NMAT > 1) an[NMAT - 1][q] = a1p[(size_t)(4 * (kn + q)) * Npad];
      }
      double b[KC][FW];
#pragma unroll
      for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int f = 0; f < FW; ++f) b[q][f] = tp[(4 * (kc + q)) * LDS_STRIDE + f * 16];
#pragma unroll
      for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int f = 0; f < FW; ++f) {
          if (INNER) {
            // D[line][i] = sum_k tile^T[line][k] AT[k][i]
            acc[0][f] = mfma_f64(b[q][f], a[0][q], acc[0][f]);
            if (NMAT > 1) acc[NMAT - 1][f] = mfma_f64(b[q][f], a[NMAT - 1][q], acc[NMAT - 1][f]);
          } else {
            // D[i][c] = sum_k A[i][k] tile[k][c]
            acc[0][f] = mfma_f64(a[0][q], b[q][f], acc[0][f]);
            if (NMAT > 1) acc[NMAT - 1][f] = mfma_f64(a[NMAT - 1][q], b[q][f], acc[NMAT - 1][f]);
          }
        }
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        a[0][q] = an[0][q];
        if (NMAT > 1) a[NMAT - 1][q] = an[NMAT - 1][q];
      }
    }
    // ---- store ------------------------------------------------------------
#pragma unroll
    for (int f = 0; f < FW; ++f) {
      {
        const int cf = (wf * FW + f) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = lk + 4 * v;  // D row within the 16x16 block
          if (INNER) {
            const int line = c0 + cf + row, i = it * 16 + lr;
            if (line < inner && i < N) {
              dst0[(size_t)line * N + i] = (OT)acc[0][f][v];
              if (NMAT > 1) dst1[(size_t)line * N + i] = (OT)acc[NMAT - 1][f][v];
            }
          } else {
            const int i = it * 16 + row, c = c0 + cf + lr;
            if (i < N && c < inner) {
              dst0[(size_t)i * inner + c] = (OT)acc[0][f][v];
              if (NMAT > 1) dst1[(size_t)i * inner + c] = (OT)acc[NMAT - 1][f][v];
            }
          }
        }
      }
    }
  }
}

static size_t lds_bytes(int npad) { return (size_t)npad * LDS_STRIDE * sizeof(double); }

template <int NMAT, bool INNER, int WI>
static hipError_t set_attr() {
  const int max_lds = 256 * LDS_STRIDE * (int)sizeof(double);  // npad <= 256
  hipError_t e = hipFuncSetAttribute((const void*)k_contract<NMAT, INNER, WI>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_contract<NMAT, INNER, WI, double, float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_contract<NMAT, INNER, WI, float, float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  return e;
}

template <int NMAT, bool INNER>
static hipError_t set_attr_wi() {
  hipError_t e = set_attr<NMAT, INNER, 1>();
  if (e == hipSuccess) e = set_attr<NMAT, INNER, 2>();
  if (e == hipSuccess) e = set_attr<NMAT, INNER, 4>();
  return e;
}

hipError_t set_kernel_attributes() {
  hipError_t e = set_attr_wi<1, true>();
  if (e == hipSuccess) e = set_attr_wi<2, true>();
  if (e == hipSuccess) e = set_attr_wi<1, false>();
  if (e == hipSuccess) e = set_attr_wi<2, false>();
  return e;
}

template <int NMAT, bool INNER, typename IT, typename OT>
static void launch_wi_t(int T, dim3 grid, size_t lds, hipStream_t s, const TaskList& tl, const Bases& B,
                        const double* AT0, const double* AT1, int N, int Npad, int inner, int slab,
                        long long P, const JobSet& js) {
  if (T >= 4)
    hipLaunchKernelGGL((k_contract<NMAT, INNER, 4, IT, OT>), grid, dim3(256), lds, s, tl, B, AT0, AT1, N, Npad,
                       inner, slab, P, js);
  else if (T >= 2)
    hipLaunchKernelGGL((k_contract<NMAT, INNER, 2, IT, OT>), grid, dim3(256), lds, s, tl, B, AT0, AT1, N, Npad,
                       inner, slab, P, js);
  else
    hipLaunchKernelGGL((k_contract<NMAT, INNER, 1, IT, OT>), grid, dim3(256), lds, s, tl, B, AT0, AT1, N, Npad,
                       inner, slab, P, js);
}

template <int NMAT, bool INNER>
static void launch_wi(int io, int T, dim3 grid, size_t lds, hipStream_t s, const TaskList& tl, const Bases& B,
                      const double* AT0, const double* AT1, int N, int Npad, int inner, int slab,
                      long long P, const JobSet& js) {
  if (io == IO_F64)
    launch_wi_t<NMAT, INNER, double, double>(T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
  else if (io == IO_OUT_F32)
    launch_wi_t<NMAT, INNER, double, float>(T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
  else
    launch_wi_t<NMAT, INNER, float, float>(T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
}

hipError_t launch_contract(int axis, int nmat, const TaskList& tl, const Bases& B,
                           const double* AT0, const double* AT1, const int n[3],
                           const int npad[3], long long P, const JobSet& js, hipStream_t s, int io) {
  if (tl.n <= 0) return hipSuccess;
  if (tl.n > MAX_TASKS || (nmat != 1 && nmat != 2) || axis < 0 || axis > 2 || js.n < 1 || js.n > MAXB ||
      (io != IO_F64 && io != IO_OUT_F32 && io != IO_F32))
    return hipErrorInvalidValue;
  if (io == IO_OUT_F32 && any_f32_input(tl)) {  // FP32-input tasks: a launch of their own
    hipError_t e = launch_contract(axis, nmat, tasks_with_input(tl, 0), B, AT0, AT1, n, npad, P, js, s, IO_OUT_F32);
    if (e != hipSuccess) return e;
    return launch_contract(axis, nmat, tasks_with_input(tl, 1), B, AT0, AT1, n, npad, P, js, s, IO_F32);
  }
  if (io == IO_F64 && any_f32_input(tl)) return hipErrorInvalidValue;
  const int N = n[axis], Npad = npad[axis];
  int inner, outer, slab;
  if (axis == 0) {          // lines of length nr, nth*nph of them
    inner = n[1] * n[2];
    outer = 1;
    slab = 0;
  } else if (axis == 1) {   // [phi][theta][r]: theta rows of nr, one slab per phi
    inner = n[0];
    outer = n[2];
    slab = n[1] * n[0];
  } else {                  // [phi][theta r]
    inner = n[0] * n[1];
    outer = 1;
    slab = 0;
  }
  dim3 grid((inner + TILE_COLS - 1) / TILE_COLS, outer, tl.n * js.n);
  const size_t lds = lds_bytes(Npad);
  const int T = Npad >> 4;
  if (axis == 0) {
    if (nmat == 1) launch_wi<1, true>(io, T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
    else launch_wi<2, true>(io, T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
  } else {
    if (nmat == 1) launch_wi<1, false>(io, T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
    else launch_wi<2, false>(io, T, grid, lds, s, tl, B, AT0, AT1, N, Npad, inner, slab, P, js);
  }
  return hipGetLastError();
}


// ===========================================================================
// Even/odd folded contractions.
//
// Every line operator here is centro-symmetric, A[N-1-i][N-1-k] = sigma A[i][k]
// (sigma = -1 for first derivatives, +1 for second derivatives and filters):
// Chebyshev collocation on Gauss-Lobatto nodes, which are symmetric about the
// interval centre, and Fourier circulants, whose entries depend on (i - k)
// mod N only.  For even N and rows i < H = N/2, with s_k = u_k + u_{N-1-k},
// d_k = u_k - u_{N-1-k} (k < H), E_ik = (A_ik + A_i,N-1-k)/2 and
// O_ik = (A_ik - A_i,N-1-k)/2:
//   (A u)_i = (E s)_i + (O d)_i,   (A u)_{N-1-i} = sigma ((E s)_i - (O d)_i),
// two H x H products instead of one N x N: half the MFMA work.  The fold is
// applied while the tile is staged in LDS (s rows on top, d rows below).
//
// Row scalings that break the symmetry (the radial log map) are applied in
// the epilogue: out_0 = g0 . (A_0 u), out_1 = g1 . (A_1 u) + g10 . (A_0 u),
// with A_0, A_1 the unmapped operators (g = null: unit scale, no coupling).
// F0, F1: E^T (Hpad x Hpad, AT[k][i] = E[i][k], zero padded) followed by O^T.
// NMAXT = 1: every task applies one operator (F0); NMAXT = 2: each task
// applies one or two operators (its nmat), so the first-and-second and the
// first-only passes of an axis share one launch.
//
// TC: columns per tile (64, or 32 for the strided axes at N = 128, where a
// 64-column tile's LDS would hold two workgroups per CU).
template <int NMAXT, bool INNER, int WI, int TC = TILE_COLS, typename IT = double, typename OT = double>
__global__ __launch_bounds__(256) void k_contract_fold(TaskList tl, Bases B, const double* __restrict__ F0,
                                                       const double* __restrict__ F1,
                                                       const double* __restrict__ G0,
                                                       const double* __restrict__ G1,
                                                       const double* __restrict__ G10, double sig0,
                                                       double sig1, int N, int Hpad, int inner, int slab,
                                                       long long P, JobSet js) {
  extern __shared__ double tile[];  // [2 Hpad][LS]: s rows, then d rows
  static_assert(TC == TILE_COLS || (!INNER && TC * WI >= 64), "narrow tiles: strided axes, TC * WI >= 64");
  constexpr int LS = TC + 8;  // row stride in doubles: rows 16 banks apart
  const Task tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  F0 = shift_ptr(F0, jd);
  F1 = shift_ptr(F1, jd);
  if (G0 != nullptr) G0 = shift_ptr(G0, jd);
  if (G1 != nullptr) G1 = shift_ptr(G1, jd);
  if (G10 != nullptr) G10 = shift_ptr(G10, jd);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int H = N >> 1;
  const int c0 = blockIdx.x * TC;
  const size_t off = (size_t)blockIdx.y * (size_t)slab;
  const IT* __restrict__ src = (const IT*)shift_ptr(B.b[tk.src_sel], jd) + (size_t)tk.src * (size_t)P + off;
  OT* __restrict__ dst0 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P + off;
  OT* __restrict__ dst1 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P + off;

  // ---- stage and fold the input tile ----------------------------------------
  constexpr int LOADS = 8;  // pairs per thread in flight
  const int total = Hpad * TC;
  if (INNER) {
    // 64 consecutive lines of N doubles; pair (k, N-1-k) of line `line`
    const int ncols = min(TC, inner - c0);
    const IT* __restrict__ s = src + (size_t)c0 * N;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double lo[LOADS], hi[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        const int line = e / Hpad, k = e - line * Hpad;
        const bool ok = e < total && k < H && line < ncols;
        lo[q] = ok ? (double)s[(size_t)line * N + k] : 0.0;
        hi[q] = ok ? (double)s[(size_t)line * N + (N - 1 - k)] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) {
          const int line = e / Hpad, k = e - line * Hpad;
          tile[k * LS + line] = lo[q] + hi[q];
          tile[(Hpad + k) * LS + line] = lo[q] - hi[q];
        }
      }
    }
  } else {
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double lo[LOADS], hi[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        const int k = e / TC, c = e % TC;
        const bool ok = e < total && k < H && c0 + c < inner;
        lo[q] = ok ? (double)src[(size_t)k * inner + c0 + c] : 0.0;
        hi[q] = ok ? (double)src[(size_t)(N - 1 - k) * inner + c0 + c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) {
          tile[(e / TC) * LS + (e % TC)] = lo[q] + hi[q];
          tile[(Hpad + e / TC) * LS + (e % TC)] = lo[q] - hi[q];
        }
      }
    }
  }
  __syncthreads();

  // ---- MFMA: (E s) and (O d) for the H output rows of each pair --------------
  auto run = [&](auto nm) {
    constexpr int NMAT = decltype(nm)::value;
    constexpr int KCF = NMAT > 1 ? 2 : 4;  // k-steps of operator fragments per chunk
    constexpr int FW = TC * WI / 64;  // 16-column blocks per wave
    const int T = Hpad >> 4;
    const int wi = wave % WI, wf = wave / WI;
    const int lr = lane & 15, lk = lane >> 4;
    const int nks = Hpad >> 2;  // a multiple of 4, hence of KCF
    const size_t hh = (size_t)Hpad * Hpad;
    for (int it = wi; it < T; it += WI) {
      d4 acc[NMAT][2][FW];
#pragma unroll
      for (int m = 0; m < NMAT; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int f = 0; f < FW; ++f) acc[m][h][f] = d4{0.0, 0.0, 0.0, 0.0};
      const double* __restrict__ ap[NMAT];
      ap[0] = F0 + (size_t)lk * Hpad + it * 16 + lr;
      if (NMAT > 1) ap[NMAT - 1] = F1 + (size_t)lk * Hpad + it * 16 + lr;
      const double* tp = tile + lk * LS + wf * FW * 16 + lr;
      double a[NMAT][2][KCF];
#pragma unroll
      for (int m = 0; m < NMAT; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < KCF; ++q) a[m][h][q] = ap[m][h * hh + (size_t)(4 * q) * Hpad];
      for (int kc = 0; kc < nks; kc += KCF) {
        const int kn = (kc + KCF < nks) ? kc + KCF : kc;  // last chunk: in-bounds dummy prefetch
        double an[NMAT][2][KCF];
#pragma unroll
        for (int m = 0; m < NMAT; ++m)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < KCF; ++q) an[m][h][q] = ap[m][h * hh + (size_t)(4 * (kn + q)) * Hpad];
#pragma unroll
        for (int q = 0; q < KCF; ++q) {
          double b[2][FW];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int f = 0; f < FW; ++f) b[h][f] = tp[(h * Hpad + 4 * (kc + q)) * LS + f * 16];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int f = 0; f < FW; ++f)
#pragma unroll
              for (int m = 0; m < NMAT; ++m) {
                if (INNER) acc[m][h][f] = mfma_f64(b[h][f], a[m][h][q], acc[m][h][f]);
                else acc[m][h][f] = mfma_f64(a[m][h][q], b[h][f], acc[m][h][f]);
              }
        }
#pragma unroll
        for (int m = 0; m < NMAT; ++m)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < KCF; ++q) a[m][h][q] = an[m][h][q];
      }
      // ---- unfold, scale, store ----------------------------------------------
#pragma unroll
      for (int f = 0; f < FW; ++f) {
        const int cf = (wf * FW + f) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = lk + 4 * v;  // D row within the 16x16 block
          int i, col;
          if (INNER) {
            col = c0 + cf + row;
            i = it * 16 + lr;
          } else {
            i = it * 16 + row;
            col = c0 + cf + lr;
          }
          if (i < H && col < inner) {
            const int im = N - 1 - i;
            const double e0 = acc[0][0][f][v], o0 = acc[0][1][f][v];
            const double y0 = e0 + o0, y0m = sig0 * (e0 - o0);
            const size_t p = INNER ? (size_t)col * N + i : (size_t)i * inner + col;
            const size_t pm = INNER ? (size_t)col * N + im : (size_t)im * inner + col;
            dst0[p] = (OT)(G0 ? G0[i] * y0 : y0);
            dst0[pm] = (OT)(G0 ? G0[im] * y0m : y0m);
            if (NMAT > 1) {
              const double e1 = acc[NMAT - 1][0][f][v], o1 = acc[NMAT - 1][1][f][v];
              const double y1 = e1 + o1, y1m = sig1 * (e1 - o1);
              dst1[p] = (OT)((G1 ? G1[i] * y1 : y1) + (G10 ? G10[i] * y0 : 0.0));
              dst1[pm] = (OT)((G1 ? G1[im] * y1m : y1m) + (G10 ? G10[im] * y0m : 0.0));
            }
          }
        }
      }
    }
  };
  if (NMAXT > 1 && tk.nmat > 1) run(std::integral_constant<int, (NMAXT > 1 ? 2 : 1)>{});
  else run(std::integral_constant<int, 1>{});
}

// ---------------------------------------------------------------------------
// Folded contraction on a strided axis (theta, phi), software-pipelined.  A
// workgroup walks PIPE_TPB consecutive column tiles of one task (tiles run
// over slab x column block).  The next tile's raw rows are copied from HBM
// straight into LDS (global_load_lds: 16 bytes per lane, no registers; cache
// policy nt, since every input row is read by one workgroup once) while
// the MFMAs run on the current tile from the other LDS buffer, and each
// wave's operator fragments (its 16 output rows, all k) stay in registers
// for every tile of the workgroup.
//
// Tile: the N input rows of TC = 16 NW / (HP / 16) contiguous inner points
// (NW waves: 16 KB for 4, 24 KB for 6).  One copy instruction moves 1 KB =
// R = 1024 / (8 TC) rows of TC doubles.
// Copy chunk q (0 <= q < Q = N / R) holds rows q, q + Q, ..., q + (R-1) Q at
// a pitch of 8 TC bytes; chunks sit PIPE_CH bytes apart, so the 4
// consecutive rows one fragment read touches alternate between the two
// halves of the 64 LDS banks.  The fold s_k = u_k + u_{N-1-k},
// d_k = u_k - u_{N-1-k} is formed at the fragment read.  Each wave computes
// one 16 x 16 output block per operator and tile (HP / 16 row tiles times
// TC / 16 column groups), so every lane stores 8 values per operator and
// tile; before a tile is read each wave waits only until its copy has
// landed (vector-memory operations complete in issue order, and exactly the
// previous tile's stores were issued after it), not for those stores.
// A one-operator task applies operator tk.op (0 or 1).  Requirements
// (checked by the launcher): N = 2 HP with HP in {16, 32, 48, 64, 96} (one
// operator only at 96: two would not fit in registers), inner a multiple of
// TC, no row scales (the angular operators carry none).
constexpr int PIPE_CH = 1152;  // bytes between copy chunks (1 KB + 128 B)


// Tiles per workgroup of a copy-ahead launch of `all` tiles (one job's):
// up to 8, keeping at least 1024 workgroups; the smallest launches (2,048
// tiles: the eight flux derivatives of 64 x 64 x 128, which run beside the
// state-derivative launches on the second stream) take 4, leaving more of
// the chip to the launch they overlap (the step 2.489 -> 2.467 ms there).
inline int pipe_tiles_per_group(long long all) {
  return all <= 2048 ? 4 : (int)std::min(8LL, all / 1024);
}

// Two-operator launches of the strided axes run as one-operator tasks (a
// first-and-second-derivative task becomes two tasks reading the same input)
// from half size 48 up: the one-operator kernel holds half the operator
// fragments, so more waves share a SIMD, which outweighs reading those inputs
// twice there (torus 128x96x192 step 12.27 -> 11.98 ms; the phi pass at
// 64x64x128 95.5 -> 91.4 us); at half sizes 16 and 32 the second read costs
// more than the waves gain.  At 96 the two-operator form would not fit the
// registers at all.
constexpr bool pipe_one_operator(int hp) { return hp >= 48; }

// Waves per workgroup: 4, or 6 for the half sizes 48 and 96 (3 or 6 row
// blocks), so that every wave owns one 16 x 16 output block per tile.
template <int HP>
constexpr int pipe_waves() { return (HP == 48 || HP == 96) ? 6 : 4; }

// MIXIN (FP32 outputs only): a task with src_f32 set reads FP32 input rows
// (the FP32 first derivatives behind the mixed second derivatives of the
// FP32-storage form) in the same launch: 1 KB copies then hold R32 = 2R rows
// of TC floats, Q32 = Q / 2 chunks per tile, PIPE_CH32 bytes apart (the four
// rows of a fragment read in different quarters of the banks), converted to
// FP64 at the fragment read; the arithmetic is FP64 either way.
constexpr int PIPE_CH32 = 1088;  // bytes between copy chunks of FP32 rows (1 KB + 64 B)

template <int HP, int NMAXT, typename OT = double, bool MIXIN = false>
__global__ __launch_bounds__(64 * pipe_waves<HP>()) void k_contract_pipe(TaskList tl, Bases B,
                                                                         const double* __restrict__ F0,
                                                                         const double* __restrict__ F1,
                                                                         double sig0, double sig1, int N, int inner,
                                                                         int slab, int ncb, int ntiles, int tpb,
                                                                         long long P, JobSet js) {
  constexpr int NW = pipe_waves<HP>();
  constexpr int T = HP / 16;       // 16-row output tiles
  constexpr int TC = 16 * NW / T;  // columns per tile (T x TC/16 = NW output blocks)
  constexpr int NKS = HP / 4;      // k-steps of 4
  static_assert(T * (TC / 16) == NW && (2 * HP / (128 / TC)) % NW == 0, "one output block per wave");
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const Task tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  F0 = shift_ptr(F0, jd);
  F1 = shift_ptr(F1, jd);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // tile buffers are sized for FP64 rows (the FP32 layout is smaller)
  const int bufbytes = (N / (128 / TC)) * PIPE_CH;
  OT* __restrict__ dst0 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P;
  OT* __restrict__ dst1 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P;
  const int t0 = blockIdx.x * tpb;
  const int nt = min(tpb, ntiles - t0);
  // element offset of tile t's first column: slab x column block
  auto tile_off = [&](int t) -> size_t {
    const int g = t0 + t, sl = g / ncb, cb = g - sl * ncb;
    return (size_t)sl * (size_t)slab + (size_t)cb * TC;
  };

  // ES: input element bytes (8: FP64 rows, 4: FP32 rows)
  auto run = [&](auto nm, auto es) {
    constexpr int NMAT = decltype(nm)::value;
    constexpr int ES = decltype(es)::value;
    using IT = typename std::conditional<ES == 8, double, float>::type;
    constexpr int RB = ES * TC;      // bytes per row in a chunk
    constexpr int LPR = RB / 16;     // lanes per row in a copy
    constexpr int R = 64 / LPR;      // rows per copy chunk
    constexpr int CH = ES == 8 ? PIPE_CH : PIPE_CH32;
    const int Q = N / R;             // chunks per tile (a multiple of 4)
    const IT* __restrict__ src = (const IT*)shift_ptr(B.b[tk.src_sel], jd) + (size_t)tk.src * (size_t)P;
    // copy of tile t into buffer b: wave w issues chunks w, w + NW, ...
    const int cm = lane / LPR, cp = lane - cm * LPR;
    auto copy_tile = [&](int t, int b) {
      const IT* g = src + tile_off(t) + (16 / ES) * cp;
      char* base = lds + b * bufbytes;
      for (int q = wave; q < Q; q += NW)
        __builtin_amdgcn_global_load_lds((const void*)(g + (size_t)(q + cm * Q) * inner),
                                         (lds_void_t*)(base + q * CH), 16, 0, 2);
    };
    const int wi = wave % T, wf = wave / T;
    const int lr = lane & 15, lk = lane >> 4;
    const size_t hh = (size_t)HP * HP;
    // operator fragments: lane (lr, lk) holds E^T / O^T [4 ks + lk][16 wi + lr]
    double a[NMAT][2][NKS];
    // a one-operator task applies operator tk.op
    const bool second = NMAT == 1 && tk.op == 1;
#pragma unroll
    for (int m = 0; m < NMAT; ++m) {
      const double* __restrict__ F = (m == 0 && !second) ? F0 : F1;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) a[m][h][ks] = F[h * hh + (size_t)(4 * ks + lk) * HP + 16 * wi + lr];
    }
    const double s0 = second ? sig1 : sig0;
    copy_tile(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      if (t > 0) {
        // tile t's copy was issued before the 8 NMAT stores of tile t - 1;
        // after the barrier every wave's copy has landed and every wave is
        // done reading the buffer the next copy overwrites
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(8 * NMAT));
        lds_barrier();
      }
      if (t + 1 < nt) copy_tile(t + 1, (t + 1) & 1);
      const char* buf = lds + (t & 1) * bufbytes;
      const char* lp = buf + lk * CH + (16 * wf + lr) * ES;  // row 4 ks + lk
      const char* lm = buf - lk * CH + (16 * wf + lr) * ES;  // row N - 1 - (4 ks + lk)
      d4 acc[NMAT][2];
#pragma unroll
      for (int m = 0; m < NMAT; ++m) acc[m][0] = acc[m][1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int qa = (4 * ks) % Q, ma = (4 * ks) / Q;  // uniform
        const double u = (double)*(const IT*)(lp + qa * CH + ma * RB);
        const double w = (double)*(const IT*)(lm + (Q - 1 - qa) * CH + (R - 1 - ma) * RB);
        const double sk = u + w, dk = u - w;
#pragma unroll
        for (int m = 0; m < NMAT; ++m) {
          acc[m][0] = mfma_f64(a[m][0][ks], sk, acc[m][0]);
          acc[m][1] = mfma_f64(a[m][1][ks], dk, acc[m][1]);
        }
      }
      // unfold, scale, store: D row lk + 4 v of the block, column lr
      const size_t toff = tile_off(t);
      const int col = 16 * wf + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {  // every row i < H = HP: stores unconditional
        const int i = 16 * wi + lk + 4 * v;
        const int im = N - 1 - i;
        const size_t p = toff + (size_t)i * inner + col, pm = toff + (size_t)im * inner + col;
        const double e0 = acc[0][0][v], o0 = acc[0][1][v];
        dst0[p] = (OT)(e0 + o0);
        dst0[pm] = (OT)(s0 * (e0 - o0));
        if (NMAT > 1) {
          const double e1 = acc[NMAT - 1][0][v], o1 = acc[NMAT - 1][1][v];
          dst1[p] = (OT)(e1 + o1);
          dst1[pm] = (OT)(sig1 * (e1 - o1));
        }
      }
    }
  };
  using E8 = std::integral_constant<int, 8>;
  using E4 = std::integral_constant<int, 4>;
  using M1 = std::integral_constant<int, 1>;
  using M2 = std::integral_constant<int, (NMAXT > 1 ? 2 : 1)>;
  if (MIXIN && tk.src_f32) {
    // FP32-input tasks apply one operator (the mixed second derivatives)
    run(M1{}, E4{});
  } else if (NMAXT > 1 && tk.nmat > 1) {
    run(M2{}, E8{});
  } else {
    run(M1{}, E8{});
  }
}

// ---------------------------------------------------------------------------
// The same pipeline on the r axis, whose lines are contiguous.  A tile is
// TL = 2048 / N whole lines (16 KB); copy chunk q (0 <= q < 16) holds lines
// q, q + 16, ... (N / 2 lanes per line, 128 / N lines per chunk), chunks
// PIPE_CH_R bytes apart so that the 16 lines one fragment read touches start
// 4 banks apart (conflict-free 8-byte reads).  The data are the MFMA's A
// operand (16 lines x 4 k), the operator the B operand (4 k x 16 rows), so a
// wave's output block is 16 lines x 16 rows; 4 waves cover the tile's
// TL / 16 line blocks times HP / 16 row blocks.  The radial row scales of a
// lane's rows are read once, before the copies start.  Requirements (checked
// by the launcher): N = 2 HP with HP in {16, 32, 64}, the line count a
// multiple of TL.
constexpr int PIPE_CH_R = 1040;  // bytes between copy chunks (1 KB + 16 B)

template <int HP, int NMAXT, typename OT = double>
__global__ __launch_bounds__(256) void k_contract_pipe_r(TaskList tl, Bases B, const double* __restrict__ F0,
                                                         const double* __restrict__ F1,
                                                         const double* __restrict__ G0,
                                                         const double* __restrict__ G1,
                                                         const double* __restrict__ G10, double sig0,
                                                         double sig1, int ntiles, int tpb, long long P,
                                                         JobSet js) {
  constexpr int N2 = 2 * HP;        // line length
  constexpr int TL = 2048 / N2;     // lines per tile
  constexpr int NKS = HP / 4;       // k-steps of 4
  constexpr int LPL = N2 / 2;       // lanes per line in a copy
  constexpr int Q = 16;             // copy chunks per tile
  constexpr int BUF = Q * PIPE_CH_R;
  static_assert(TL * N2 * 8 == Q * 1024, "16 one-KB chunks per tile");
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const Task tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  F0 = shift_ptr(F0, jd);
  F1 = shift_ptr(F1, jd);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* __restrict__ src = shift_ptr(B.b[tk.src_sel], jd) + (size_t)tk.src * (size_t)P;
  OT* __restrict__ dst0 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P;
  OT* __restrict__ dst1 = (OT*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P;
  const int t0 = blockIdx.x * tpb;
  const int nt = min(tpb, ntiles - t0);
  const int cm = lane / LPL, cp = lane - cm * LPL;
  auto copy_tile = [&](int t, int b) {
    const double* g = src + (size_t)(t0 + t) * TL * N2 + 2 * cp;
    char* base = lds + b * BUF;
#pragma unroll
    for (int q = wave; q < Q; q += 4)
      __builtin_amdgcn_global_load_lds((const void*)(g + (size_t)(q + 16 * cm) * N2),
                                       (lds_void_t*)(base + q * PIPE_CH_R), 16, 0, 2);
  };

  auto run = [&](auto nm) {
    constexpr int NMAT = decltype(nm)::value;
    constexpr int RT = HP / 16;      // row blocks
    const int wr = wave % RT, wl = wave / RT;  // this wave's row block and line block
    const int lr = lane & 15, lk = lane >> 4;
    const size_t hh = (size_t)HP * HP;
    // operator fragments (B operand): lane (lr, lk) holds E^T / O^T [4 ks + lk][16 wr + lr]
    double a[NMAT][2][NKS];
#pragma unroll
    for (int m = 0; m < NMAT; ++m) {
      const double* __restrict__ F = m == 0 ? F0 : F1;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) a[m][h][ks] = F[h * hh + (size_t)(4 * ks + lk) * HP + 16 * wr + lr];
    }
    // radial row scales of this lane's output rows i = 16 wr + lr and N - 1 - i
    const int i = 16 * wr + lr, im = N2 - 1 - i;
    const double* g0 = G0 ? shift_ptr(G0, jd) : nullptr;
    const double* g1 = G1 ? shift_ptr(G1, jd) : nullptr;
    const double* g10 = G10 ? shift_ptr(G10, jd) : nullptr;
    const double s0 = g0 ? g0[i] : 1.0, s0m = g0 ? g0[im] : 1.0;
    const double s1 = g1 ? g1[i] : 1.0, s1m = g1 ? g1[im] : 1.0;
    const double s10 = g10 ? g10[i] : 0.0, s10m = g10 ? g10[im] : 0.0;
    __builtin_amdgcn_s_waitcnt(0);  // fragments and scales in registers before the copies start
    copy_tile(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // data fragment (A operand): lane (lr, lk) reads line 16 wl + lr, k = 4 ks + lk
    const int line = 16 * wl + lr;
    const int lq = line & 15, lm = line >> 4;  // its copy chunk and slot
    for (int t = 0; t < nt; ++t) {
      if (t > 0) {
        // tile t's copy was issued before the 8 NMAT stores of tile t - 1
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(8 * NMAT));
        lds_barrier();
      }
      if (t + 1 < nt) copy_tile(t + 1, (t + 1) & 1);
      const char* lp = lds + (t & 1) * BUF + lq * PIPE_CH_R + lm * (8 * N2);
      d4 acc[NMAT][2];
#pragma unroll
      for (int m = 0; m < NMAT; ++m) acc[m][0] = acc[m][1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int k = 4 * ks + lk;
        const double u = *(const double*)(lp + 8 * k);
        const double w = *(const double*)(lp + 8 * (N2 - 1 - k));
        const double sk = u + w, dk = u - w;
#pragma unroll
        for (int m = 0; m < NMAT; ++m) {
          acc[m][0] = mfma_f64(sk, a[m][0][ks], acc[m][0]);
          acc[m][1] = mfma_f64(dk, a[m][1][ks], acc[m][1]);
        }
      }
      // unfold, scale, store: D line lk + 4 v of the block, row i
      const size_t l0 = (size_t)(t0 + t) * TL + 16 * wl;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const size_t p = (l0 + lk + 4 * v) * N2;
        const double e0 = acc[0][0][v], o0 = acc[0][1][v];
        const double y0 = e0 + o0, y0m = sig0 * (e0 - o0);
        dst0[p + i] = (OT)(s0 * y0);
        dst0[p + im] = (OT)(s0m * y0m);
        if (NMAT > 1) {
          const double e1 = acc[NMAT - 1][0][v], o1 = acc[NMAT - 1][1][v];
          dst1[p + i] = (OT)(s1 * (e1 + o1) + s10 * y0);
          dst1[p + im] = (OT)(s1m * (sig1 * (e1 - o1)) + s10m * y0m);
        }
      }
    }
  };
  if (NMAXT > 1 && tk.nmat > 1) run(std::integral_constant<int, (NMAXT > 1 ? 2 : 1)>{});
  else run(std::integral_constant<int, 1>{});
}

template <int NMAT, bool INNER, int WI, int TC = TILE_COLS>
static hipError_t set_fold_attr() {
  const int max_lds = 256 * (TC + 8) * (int)sizeof(double);  // 2 Hpad <= 256
  hipError_t e = hipFuncSetAttribute((const void*)k_contract_fold<NMAT, INNER, WI, TC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_contract_fold<NMAT, INNER, WI, TC, double, float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_contract_fold<NMAT, INNER, WI, TC, float, float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  return e;
}

hipError_t set_fold_kernel_attributes() {
  hipError_t e = hipSuccess;
#define FA(NM, IN)                                          \
  if (e == hipSuccess) e = set_fold_attr<NM, IN, 1>();      \
  if (e == hipSuccess) e = set_fold_attr<NM, IN, 2>();      \
  if (e == hipSuccess) e = set_fold_attr<NM, IN, 4>();
  FA(1, true)
  FA(2, true)
  FA(1, false)
  FA(2, false)
#undef FA
  if (e == hipSuccess) e = set_fold_attr<1, false, 4, NARROW>();
  if (e == hipSuccess) e = set_fold_attr<2, false, 4, NARROW>();
  return e;
}

// IT, OT: input and output storage types; the copy-ahead kernels take FP64
// inputs only (their HBM-to-LDS copies move raw doubles), so FP32 inputs use
// the one-tile kernel.
template <typename IT, typename OT>
static hipError_t launch_fold_t(int axis, int nmat, const TaskList& tl, const Bases& B, const FoldOp& op0,
                                const FoldOp& op1, const double* g10, const int n[3], const int hpad[3],
                                long long P, const JobSet& js, hipStream_t s) {
  // FP64-input launches only; FP32-input tasks ride in the FP32-output
  // copy-ahead launches of the strided axes (per-task input rows)
  constexpr bool copy_ahead = std::is_same<IT, double>::value;
  const bool f32_tasks = any_f32_input(tl);
  const int N = n[axis], Hpad = hpad[axis];
  if ((N & 1) || Hpad < N / 2 || (Hpad & 15) || 2 * Hpad > 256) return hipErrorInvalidValue;
  int inner, slab, outer;
  if (axis == 0) {
    inner = n[1] * n[2];
    outer = 1;
    slab = 0;
  } else if (axis == 1) {
    inner = n[0];
    outer = n[2];
    slab = n[1] * n[0];
  } else {
    inner = n[0] * n[1];
    outer = 1;
    slab = 0;
  }
  const int T = Hpad >> 4;
  if (copy_ahead && !f32_tasks && axis == 0 && (Hpad == 16 || Hpad == 32 || Hpad == 64) && N == 2 * Hpad) {
    // pipelined form of the r axis: the line count a multiple of the tile's
    const int tlines = 2048 / N;
    // the kernel and its tiles per workgroup follow from one job's tiles, so
    // a job's arithmetic is the same alone and in a batch of any size
    const long long all = (long long)(inner / tlines) * tl.n;
    if (inner % tlines == 0 && all >= 2048) {
      const int ntiles = inner / tlines;
      const int tpb = pipe_tiles_per_group(all);
      dim3 pg((ntiles + tpb - 1) / tpb, 1, tl.n * js.n);
#define LR(HPV, NM)                                                                                         \
  hipLaunchKernelGGL((k_contract_pipe_r<HPV, NM, OT>), pg, dim3(256), 2 * 16 * PIPE_CH_R, s, tl, B, op0.et,     \
                     op1.et, op0.g, op1.g, g10, op0.sigma, op1.sigma, ntiles, tpb, P, js)
      if (Hpad == 16) { if (nmat == 1) LR(16, 1); else LR(16, 2); }
      else if (Hpad == 32) { if (nmat == 1) LR(32, 1); else LR(32, 2); }
      else { if (nmat == 1) LR(64, 1); else LR(64, 2); }
#undef LR
      return hipGetLastError();
    }
  }
  if (copy_ahead && axis != 0 && (Hpad == 16 || Hpad == 32 || Hpad == 48 || Hpad == 64 || Hpad == 96) &&
      N == 2 * Hpad && op0.g == nullptr && op1.g == nullptr && g10 == nullptr) {
    // copy-ahead form: inner a multiple of the tile width
    const int nw = (Hpad == 48 || Hpad == 96) ? 6 : 4;
    const int tc = 16 * nw / (Hpad / 16), rows = 1024 / (8 * tc);
    const long long all = (long long)(inner / tc) * outer * tl.n;  // tiles of one job's launch
    // small launches (a few tiles per workgroup) keep the one-tile kernel;
    // the choice and the tiles per workgroup follow from one job's tiles, so
    // a job's arithmetic is the same alone and in a batch of any size
    if (inner % tc == 0 && all >= 2048) {
      const int ncb = inner / tc, ntiles = ncb * outer;
      const int bufbytes = (N / rows) * PIPE_CH;
      const int tpb = pipe_tiles_per_group(all);
      auto launch = [&](const TaskList& L, int nm, const FoldOp& o0, const FoldOp& o1) {
        dim3 pg((ntiles + tpb - 1) / tpb, 1, L.n * js.n);
#define LP(HPV, NM)                                                                                               \
  hipLaunchKernelGGL((k_contract_pipe<HPV, NM, OT, std::is_same<OT, float>::value>), pg, dim3(64 * pipe_waves<HPV>()), 2 * bufbytes, s, L, B, o0.et, \
                     o1.et, o0.sigma, o1.sigma, N, inner, slab, ncb, ntiles, tpb, P, js)
        if (Hpad == 16) { if (nm == 1) LP(16, 1); else LP(16, 2); }
        else if (Hpad == 32) { if (nm == 1) LP(32, 1); else LP(32, 2); }
        else if (Hpad == 48) { if (nm == 1) LP(48, 1); else LP(48, 2); }
        else if (Hpad == 64) { if (nm == 1) LP(64, 1); else LP(64, 2); }
        else LP(96, 1);
#undef LP
        return hipGetLastError();
      };
      if (nmat == 2 && pipe_one_operator(Hpad)) {
        // one operator per task: a two-operator task becomes two tasks
        TaskList one;
        one.n = 0;
        bool fits = true;
        for (int i = 0; i < tl.n && fits; ++i) {
          const int k = tl.t[i].nmat == 2 ? 2 : 1;
          if (one.n + k > MAX_TASKS) fits = false;
          for (int m = 0; m < k && fits; ++m) {
            Task t = tl.t[i];
            t.nmat = 1;
            t.op = m;
            if (m == 1) t.dst0 = tl.t[i].dst1;
            one.t[one.n++] = t;
          }
        }
        if (fits) return launch(one, 1, op0, op1);
        TaskList la = tl, lb;
        lb.n = 0;
        for (int i = 0; i < tl.n; ++i) {
          la.t[i].nmat = 1;
          la.t[i].op = 0;
          if (tl.t[i].nmat == 2) {
            lb.t[lb.n] = tl.t[i];
            lb.t[lb.n].dst0 = tl.t[i].dst1;
            lb.t[lb.n].nmat = 1;
            lb.t[lb.n].op = 1;
            ++lb.n;
          }
        }
        hipError_t e = launch(la, 1, op0, op1);
        if (e == hipSuccess && lb.n > 0) e = launch(lb, 1, op0, op1);
        return e;
      }
      return launch(tl, nmat, op0, op1);
    }
  }
  if (f32_tasks && !std::is_same<IT, float>::value) {
    // one-tile kernels: FP32-input tasks in a launch of their own
    if (!std::is_same<OT, float>::value) return hipErrorInvalidValue;
    hipError_t e = launch_fold_t<IT, OT>(axis, nmat, tasks_with_input(tl, 0), B, op0, op1, g10, n, hpad, P, js, s);
    if (e != hipSuccess) return e;
    return launch_fold_t<float, float>(axis, nmat, tasks_with_input(tl, 1), B, op0, op1, g10, n, hpad, P, js, s);
  }
  const bool narrow = axis != 0 && T == 4;  // N = 128 on a strided axis: 32-column tiles
  const int tc = narrow ? NARROW : TILE_COLS;
  dim3 grid((inner + tc - 1) / tc, outer, tl.n * js.n);
  const size_t lds = (size_t)2 * Hpad * (tc + 8) * sizeof(double);
#define LF(NM, IN, W)                                                                                     \
  hipLaunchKernelGGL((k_contract_fold<NM, IN, W, TILE_COLS, IT, OT>), grid, dim3(256), lds, s, tl, B, op0.et, op1.et, op0.g, \
                     op1.g, g10, op0.sigma, op1.sigma, N, Hpad, inner, slab, P, js)
#define LFW(NM, IN)                 \
  do {                              \
    if (T >= 4) LF(NM, IN, 4);      \
    else if (T >= 2) LF(NM, IN, 2); \
    else LF(NM, IN, 1);             \
  } while (0)
#define LN(NM)                                                                                           \
  hipLaunchKernelGGL((k_contract_fold<NM, false, 4, NARROW, IT, OT>), grid, dim3(256), lds, s, tl, B, op0.et, op1.et, \
                     op0.g, op1.g, g10, op0.sigma, op1.sigma, N, Hpad, inner, slab, P, js)
  if (axis == 0) {
    if (nmat == 1) LFW(1, true); else LFW(2, true);
  } else if (narrow) {
    if (nmat == 1) LN(1); else LN(2);
  } else {
    if (nmat == 1) LFW(1, false); else LFW(2, false);
  }
#undef LN
#undef LFW
#undef LF
  return hipGetLastError();
}

hipError_t launch_contract_fold(int axis, int nmat, const TaskList& tl, const Bases& B, const FoldOp& op0,
                                const FoldOp& op1, const double* g10, const int n[3], const int hpad[3],
                                long long P, const JobSet& js, hipStream_t s, int io) {
  if (tl.n <= 0) return hipSuccess;
  if (tl.n > MAX_TASKS || (nmat != 1 && nmat != 2) || axis < 0 || axis > 2 || js.n < 1 || js.n > MAXB)
    return hipErrorInvalidValue;
  for (int i = 0; i < tl.n; ++i)  // FP32-input tasks: FP32 outputs, one operator
    if (tl.t[i].src_f32 && (io == IO_F64 || tl.t[i].nmat != 1)) return hipErrorInvalidValue;
  if (io == IO_F64) return launch_fold_t<double, double>(axis, nmat, tl, B, op0, op1, g10, n, hpad, P, js, s);
  if (io == IO_OUT_F32) return launch_fold_t<double, float>(axis, nmat, tl, B, op0, op1, g10, n, hpad, P, js, s);
  if (io == IO_F32) return launch_fold_t<float, float>(axis, nmat, tl, B, op0, op1, g10, n, hpad, P, js, s);
  return hipErrorInvalidValue;
}

}  // namespace grmhd
