// Reduced-precision derivative contractions (the mixed-precision form):
// the same dense line contractions as contract.hip, with FP32 outputs, in
//   FP32   : v_mfma_f32_16x16x4f32, FP32 operands and accumulation;
//   BF16x3 : v_mfma_f32_16x16x32_bf16 on split operands x = x_hi + x_lo
//            (bf16 each), A x ~ A_hi x_hi + A_hi x_lo + A_lo x_hi, FP32
//            accumulation.
// Before the cast every grid line is shifted by its value at the middle node,
// computed in FP64.  Derivative matrices annihilate constants (zero row sums),
// so the shift changes nothing in exact arithmetic and the rounding error
// scales with the variation along the line instead of its magnitude.  Inputs
// are FP64 (state, fluxes) or FP32 (first derivatives feeding the mixed
// second derivatives), chosen per task.
//
// Fragment layouts (measured on gfx950):
//   f32 16x16x4   A: lane l holds A[l%16][l/16]; B: B[l/16][l%16];
//                 D: lane l, reg v holds D[4(l/16) + v][l%16]
//   bf16 16x16x32 A: lane l holds A[l%16][8(l/16) + q], q = 0..7 (any k order
//                 shared by A and B gives the same sum); B: B[8(l/16) + q][l%16];
//                 D as for f32.
#include "grmhd_internal.h"

#include <algorithm>
#include <type_traits>

namespace grmhd {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

constexpr int MT_COLS = 64;
constexpr int F32_STRIDE = 80;   // floats per tile row: 4 rows cover 64 banks once
constexpr int BF_PAD = 8;        // bf16 padding per tile row (rows 4 banks apart)
constexpr int KC32 = 4;          // FP32 form: k-steps (of 4) of operator fragments per chunk

// Start of the task's input field (FP32 or FP64 storage).
template <class T>
__device__ __forceinline__ const T* field_base(const MixedTask& t, const Bases& B, long long P, long long jd) {
  return (const T*)shift_ptr(B.b[t.src_sel], jd) + (size_t)t.src * (size_t)P;
}

__device__ __forceinline__ double load_in(const MixedTask& t, const Bases& B, long long P,
                                          long long jd, size_t off) {
  if (t.src_f32) return (double)(((const float*)shift_ptr(B.b[t.src_sel], jd)) + (size_t)t.src * (size_t)P)[off];
  return (shift_ptr(B.b[t.src_sel], jd) + (size_t)t.src * (size_t)P)[off];
}

// Element (k, c) of the tile of this workgroup, as an offset inside one field.
// INNER: lines c0 + c of length N (r axis); otherwise rows k of `inner` points.
template <bool INNER>
__device__ __forceinline__ size_t elem(int k, int c, int c0, int N, int inner, size_t slab_off) {
  return INNER ? (size_t)(c0 + c) * N + k : slab_off + (size_t)k * inner + c0 + c;
}

// ---------------------------------------------------------------------------
template <int NMAT, bool INNER, int WI>
__global__ __launch_bounds__(256) void k_contract_f32(MixedTaskList tl, Bases B,
                                                      const float* __restrict__ AT0,
                                                      const float* __restrict__ AT1, int N, int Npad,
                                                      int inner, int slab, long long P, JobSet js) {
  extern __shared__ float tf[];  // [Npad][F32_STRIDE] + 64 doubles of line offsets
  double* shift = (double*)(tf + (size_t)Npad * F32_STRIDE);
  const MixedTask tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  AT0 = shift_ptr(AT0, jd);
  AT1 = shift_ptr(AT1, jd);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = blockIdx.x * MT_COLS;
  const size_t soff = (size_t)blockIdx.y * (size_t)slab;
  const int ncols = min(MT_COLS, inner - c0);
  if (threadIdx.x < MT_COLS)
    shift[threadIdx.x] =
        threadIdx.x < ncols ? load_in(tk, B, P, jd, elem<INNER>(N / 2, threadIdx.x, c0, N, inner, soff)) : 0.0;
  __syncthreads();
  // the input precision is uniform per task: one straight-line fill per type
  auto fill = [&](const auto* __restrict__ fsrc) {
    constexpr int LOADS = 16;
    const int total = Npad * MT_COLS;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double v[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        int k, c;
        if (INNER) { c = e / Npad; k = e - c * Npad; } else { k = e >> 6; c = e & 63; }
        v[q] = (e < total && k < N && c < ncols) ? (double)fsrc[elem<INNER>(k, c, c0, N, inner, soff)] - shift[c]
                                                 : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) {
          int k, c;
          if (INNER) { c = e / Npad; k = e - c * Npad; } else { k = e >> 6; c = e & 63; }
          tf[k * F32_STRIDE + c] = (float)v[q];
        }
      }
    }
  };
  if (tk.src_f32) fill(field_base<float>(tk, B, P, jd));
  else fill(field_base<double>(tk, B, P, jd));
  __syncthreads();
  const int T = Npad >> 4;
  constexpr int FW = WI;  // 16-column fragments per wave; WI waves along the rows
  const int wi = wave % WI, wf = wave / WI;
  const int lr = lane & 15, lk = lane >> 4;
  float* dst0 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P + soff;
  float* dst1 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P + soff;
  for (int it = wi; it < T; it += WI) {
    f4 acc[NMAT][FW];
#pragma unroll
    for (int m = 0; m < NMAT; ++m)
#pragma unroll
      for (int f = 0; f < FW; ++f) acc[m][f] = f4{0.f, 0.f, 0.f, 0.f};
    const float* a0p = AT0 + (size_t)lk * Npad + it * 16 + lr;
    const float* a1p = (NMAT > 1 ? AT1 : AT0) + (size_t)lk * Npad + it * 16 + lr;
    const float* tp = tf + lk * F32_STRIDE + wf * FW * 16 + lr;
    // operator fragments of KC k-steps in registers, the next chunk requested
    // before the current one is consumed (the last chunk re-requests itself)
    const int nks = Npad >> 2;  // a multiple of KC32 since Npad % 16 == 0
    float a[NMAT][KC32];
#pragma unroll
    for (int q = 0; q < KC32; ++q) {
      a[0][q] = a0p[(size_t)(4 * q) * Npad];
      if (NMAT > 1) a[NMAT - 1][q] = a1p[(size_t)(4 * q) * Npad];
    }
    for (int kc = 0; kc < nks; kc += KC32) {
      const int kn = (kc + KC32 < nks) ? kc + KC32 : kc;
      float an[NMAT][KC32], b[KC32][FW];
#pragma unroll
      for (int q = 0; q < KC32; ++q) {
        an[0][q] = a0p[(size_t)(4 * (kn + q)) * Npad];
        if (NMAT > 1) an[NMAT - 1][q] = a1p[(size_t)(4 * (kn + q)) * Npad];
      }
#pragma unroll
      for (int q = 0; q < KC32; ++q)
#pragma unroll
        for (int f = 0; f < FW; ++f) b[q][f] = tp[(4 * (kc + q)) * F32_STRIDE + f * 16];
#pragma unroll
      for (int q = 0; q < KC32; ++q)
#pragma unroll
        for (int f = 0; f < FW; ++f) {
          if (INNER) {
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[q][f], a[0][q], acc[0][f], 0, 0, 0);
            if (NMAT > 1)
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[q][f], a[NMAT - 1][q], acc[NMAT - 1][f], 0, 0, 0);
          } else {
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][q], b[q][f], acc[0][f], 0, 0, 0);
            if (NMAT > 1)
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[NMAT - 1][q], b[q][f], acc[NMAT - 1][f], 0, 0, 0);
          }
        }
#pragma unroll
      for (int q = 0; q < KC32; ++q) {
        a[0][q] = an[0][q];
        if (NMAT > 1) a[NMAT - 1][q] = an[NMAT - 1][q];
      }
    }
#pragma unroll
    for (int f = 0; f < FW; ++f) {
      {
        const int cf = (wf * FW + f) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 4 * lk + v;
          if (INNER) {
            const int line = c0 + cf + row, i = it * 16 + lr;
            if (line < inner && i < N) {
              dst0[(size_t)line * N + i] = acc[0][f][v];
              if (NMAT > 1) dst1[(size_t)line * N + i] = acc[NMAT - 1][f][v];
            }
          } else {
            const int i = it * 16 + row, c = c0 + cf + lr;
            if (i < N && c < inner) {
              dst0[(size_t)i * inner + c] = acc[0][f][v];
              if (NMAT > 1) dst1[(size_t)i * inner + c] = acc[NMAT - 1][f][v];
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Operators for BF16x3: row-major A[i][k] (i padded to 16, k padded to 32),
// high and low parts in two arrays.  The tile is stored column-major
// (tile[c][k], k contiguous) so each lane reads 8 consecutive k with one
// 16-byte load, for both the r axis and the theta/phi axes.
template <int NMAT, bool INNER, int WI>
__global__ __launch_bounds__(256) void k_contract_bf3(MixedTaskList tl, Bases B,
                                                      const __bf16* __restrict__ A0h,
                                                      const __bf16* __restrict__ A0l,
                                                      const __bf16* __restrict__ A1h,
                                                      const __bf16* __restrict__ A1l, int N, int Npad,
                                                      int Kpad, int inner, int slab, long long P, JobSet js) {
  extern __shared__ __bf16 tb[];  // hi [64][Kpad + BF_PAD], lo [64][Kpad + BF_PAD], 64 doubles
  const int RS = Kpad + BF_PAD;
  __bf16* thi = tb;
  __bf16* tlo = tb + (size_t)MT_COLS * RS;
  double* shift = (double*)(tb + (size_t)2 * MT_COLS * RS);
  const MixedTask tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  A0h = shift_ptr(A0h, jd);
  A0l = shift_ptr(A0l, jd);
  A1h = shift_ptr(A1h, jd);
  A1l = shift_ptr(A1l, jd);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = blockIdx.x * MT_COLS;
  const size_t soff = (size_t)blockIdx.y * (size_t)slab;
  const int ncols = min(MT_COLS, inner - c0);
  if (threadIdx.x < MT_COLS)
    shift[threadIdx.x] =
        threadIdx.x < ncols ? load_in(tk, B, P, jd, elem<INNER>(N / 2, threadIdx.x, c0, N, inner, soff)) : 0.0;
  __syncthreads();
  // the input precision is uniform per task: one straight-line fill per type
  auto fill = [&](const auto* __restrict__ fsrc) {
    constexpr int LOADS = 16;
    const int total = Kpad * MT_COLS;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double v[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        int k, c;
        if (INNER) { c = e / Kpad; k = e - c * Kpad; } else { k = e >> 6; c = e & 63; }
        v[q] = (e < total && k < N && c < ncols) ? (double)fsrc[elem<INNER>(k, c, c0, N, inner, soff)] - shift[c]
                                                 : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) {
          int k, c;
          if (INNER) { c = e / Kpad; k = e - c * Kpad; } else { k = e >> 6; c = e & 63; }
          const float x = (float)v[q];
          const __bf16 h = (__bf16)x;
          thi[c * RS + k] = h;
          tlo[c * RS + k] = (__bf16)(x - (float)h);
        }
      }
    }
  };
  if (tk.src_f32) fill(field_base<float>(tk, B, P, jd));
  else fill(field_base<double>(tk, B, P, jd));
  __syncthreads();
  const int T = Npad >> 4;
  constexpr int FW = WI;  // 16-column fragments per wave; WI waves along the rows
  const int wi = wave % WI, wf = wave / WI;
  const int lr = lane & 15, lk = lane >> 4;
  float* dst0 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P + soff;
  float* dst1 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P + soff;
  for (int it = wi; it < T; it += WI) {
    f4 acc[NMAT][FW];
#pragma unroll
    for (int m = 0; m < NMAT; ++m)
#pragma unroll
      for (int f = 0; f < FW; ++f) acc[m][f] = f4{0.f, 0.f, 0.f, 0.f};
    const size_t arow = (size_t)(it * 16 + lr) * Kpad + 8 * lk;
    for (int k0 = 0; k0 < Kpad; k0 += 32) {
      const b8 ah0 = *(const b8*)(A0h + arow + k0);
      const b8 al0 = *(const b8*)(A0l + arow + k0);
      b8 ah1 = ah0, al1 = al0;
      if (NMAT > 1) {
        ah1 = *(const b8*)(A1h + arow + k0);
        al1 = *(const b8*)(A1l + arow + k0);
      }
#pragma unroll
      for (int f = 0; f < FW; ++f) {
        {
          const int col = (wf * FW + f) * 16 + lr;
          const b8 bh = *(const b8*)(thi + col * RS + k0 + 8 * lk);
          const b8 bl = *(const b8*)(tlo + col * RS + k0 + 8 * lk);
          if (INNER) {
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, ah0, acc[0][f], 0, 0, 0);
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, ah0, acc[0][f], 0, 0, 0);
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, al0, acc[0][f], 0, 0, 0);
            if (NMAT > 1) {
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, ah1, acc[NMAT - 1][f], 0, 0, 0);
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, ah1, acc[NMAT - 1][f], 0, 0, 0);
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, al1, acc[NMAT - 1][f], 0, 0, 0);
            }
          } else {
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bh, acc[0][f], 0, 0, 0);
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bl, acc[0][f], 0, 0, 0);
            acc[0][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al0, bh, acc[0][f], 0, 0, 0);
            if (NMAT > 1) {
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bh, acc[NMAT - 1][f], 0, 0, 0);
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bl, acc[NMAT - 1][f], 0, 0, 0);
              acc[NMAT - 1][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al1, bh, acc[NMAT - 1][f], 0, 0, 0);
            }
          }
        }
      }
    }
#pragma unroll
    for (int f = 0; f < FW; ++f) {
      {
        const int cf = (wf * FW + f) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 4 * lk + v;
          if (INNER) {
            const int line = c0 + cf + row, i = it * 16 + lr;
            if (line < inner && i < N) {
              dst0[(size_t)line * N + i] = acc[0][f][v];
              if (NMAT > 1) dst1[(size_t)line * N + i] = acc[NMAT - 1][f][v];
            }
          } else {
            const int i = it * 16 + row, c = c0 + cf + lr;
            if (i < N && c < inner) {
              dst0[(size_t)i * inner + c] = acc[0][f][v];
              if (NMAT > 1) dst1[(size_t)i * inner + c] = acc[NMAT - 1][f][v];
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
static void geometry(int axis, const int n[3], int* inner, int* outer, int* slab) {
  if (axis == 0) {
    *inner = n[1] * n[2];
    *outer = 1;
    *slab = 0;
  } else if (axis == 1) {
    *inner = n[0];
    *outer = n[2];
    *slab = n[1] * n[0];
  } else {
    *inner = n[0] * n[1];
    *outer = 1;
    *slab = 0;
  }
}

size_t mixed_lds_bytes(int prec, int npad) {
  if (prec == GRMHD_MIX_FP32) return (size_t)npad * F32_STRIDE * sizeof(float) + MT_COLS * sizeof(double);
  const int kpad = round_up(npad, 32);
  return (size_t)2 * MT_COLS * (kpad + BF_PAD) * 2 + MT_COLS * sizeof(double);
}

// ---------------------------------------------------------------------------
// Folded FP32 form (even N): the even/odd split of the FP64 folded kernel
// (centro-symmetric operators, two H x H products on s_k = u_k + u_{N-1-k}
// and d_k = u_k - u_{N-1-k}).  The middle-node shift and the fold are done in
// FP64; s and d are rounded to FP32 once, the products run on FP32 MFMA.
// Row scales of the radial map are applied in the epilogue in FP64:
// out_0 = g0 . (A_0 u), out_1 = g1 . (A_1 u) + g10 . (A_0 u).
// NMAXT = 2: each task applies one or two operators (its nmat).
template <int NMAXT, bool INNER, int WI>
__global__ __launch_bounds__(256) void k_contract_f32_fold(MixedTaskList tl, Bases B, const float* __restrict__ F0,
                                                           const float* __restrict__ F1,
                                                           const double* __restrict__ G0,
                                                           const double* __restrict__ G1,
                                                           const double* __restrict__ G10, float sig0, float sig1,
                                                           int N, int Hpad, int inner, int slab, long long P,
                                                           JobSet js) {
  extern __shared__ float tf[];  // [2 Hpad][F32_STRIDE]: s rows, d rows; then 64 doubles of line offsets
  double* shift = (double*)(tf + (size_t)2 * Hpad * F32_STRIDE);
  const MixedTask tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  F0 = shift_ptr(F0, jd);
  F1 = shift_ptr(F1, jd);
  if (G0 != nullptr) G0 = shift_ptr(G0, jd);
  if (G1 != nullptr) G1 = shift_ptr(G1, jd);
  if (G10 != nullptr) G10 = shift_ptr(G10, jd);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int H = N >> 1;
  const int c0 = blockIdx.x * MT_COLS;
  const size_t soff = (size_t)blockIdx.y * (size_t)slab;
  const int ncols = min(MT_COLS, inner - c0);
  if (threadIdx.x < MT_COLS)
    shift[threadIdx.x] =
        threadIdx.x < ncols ? load_in(tk, B, P, jd, elem<INNER>(N / 2, threadIdx.x, c0, N, inner, soff)) : 0.0;
  __syncthreads();
  auto fill = [&](const auto* __restrict__ fsrc) {
    constexpr int LOADS = 8;  // pairs per thread in flight
    const int total = Hpad * MT_COLS;
    for (int e0 = threadIdx.x; e0 < total; e0 += 256 * LOADS) {
      double lo[LOADS], hi[LOADS];
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        int k, c;
        if (INNER) { c = e / Hpad; k = e - c * Hpad; } else { k = e >> 6; c = e & 63; }
        const bool ok = e < total && k < H && c < ncols;
        lo[q] = ok ? (double)fsrc[elem<INNER>(k, c, c0, N, inner, soff)] - shift[c] : 0.0;
        hi[q] = ok ? (double)fsrc[elem<INNER>(N - 1 - k, c, c0, N, inner, soff)] - shift[c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LOADS; ++q) {
        const int e = e0 + q * 256;
        if (e < total) {
          int k, c;
          if (INNER) { c = e / Hpad; k = e - c * Hpad; } else { k = e >> 6; c = e & 63; }
          tf[k * F32_STRIDE + c] = (float)(lo[q] + hi[q]);
          tf[(Hpad + k) * F32_STRIDE + c] = (float)(lo[q] - hi[q]);
        }
      }
    }
  };
  if (tk.src_f32) fill(field_base<float>(tk, B, P, jd));
  else fill(field_base<double>(tk, B, P, jd));
  __syncthreads();

  auto run = [&](auto nm) {
    constexpr int NMAT = decltype(nm)::value;
    constexpr int KCF = NMAT > 1 ? 2 : 4;
    constexpr int FW = WI;
    const int T = Hpad >> 4;
    const int wi = wave % WI, wf = wave / WI;
    const int lr = lane & 15, lk = lane >> 4;
    const int nks = Hpad >> 2;  // a multiple of 4, hence of KCF
    const size_t hh = (size_t)Hpad * Hpad;
    float* dst0 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P + soff;
    float* dst1 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P + soff;
    for (int it = wi; it < T; it += WI) {
      f4 acc[NMAT][2][FW];
#pragma unroll
      for (int m = 0; m < NMAT; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int f = 0; f < FW; ++f) acc[m][h][f] = f4{0.f, 0.f, 0.f, 0.f};
      const float* __restrict__ ap[NMAT];
      ap[0] = F0 + (size_t)lk * Hpad + it * 16 + lr;
      if (NMAT > 1) ap[NMAT - 1] = F1 + (size_t)lk * Hpad + it * 16 + lr;
      const float* tp = tf + lk * F32_STRIDE + wf * FW * 16 + lr;
      float a[NMAT][2][KCF];
#pragma unroll
      for (int m = 0; m < NMAT; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < KCF; ++q) a[m][h][q] = ap[m][h * hh + (size_t)(4 * q) * Hpad];
      for (int kc = 0; kc < nks; kc += KCF) {
        const int kn = (kc + KCF < nks) ? kc + KCF : kc;  // last chunk: in-bounds dummy prefetch
        float an[NMAT][2][KCF];
#pragma unroll
        for (int m = 0; m < NMAT; ++m)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < KCF; ++q) an[m][h][q] = ap[m][h * hh + (size_t)(4 * (kn + q)) * Hpad];
#pragma unroll
        for (int q = 0; q < KCF; ++q) {
          float b[2][FW];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int f = 0; f < FW; ++f) b[h][f] = tp[(h * Hpad + 4 * (kc + q)) * F32_STRIDE + f * 16];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int f = 0; f < FW; ++f)
#pragma unroll
              for (int m = 0; m < NMAT; ++m) {
                if (INNER) acc[m][h][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[h][f], a[m][h][q], acc[m][h][f], 0, 0, 0);
                else acc[m][h][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m][h][q], b[h][f], acc[m][h][f], 0, 0, 0);
              }
        }
#pragma unroll
        for (int m = 0; m < NMAT; ++m)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < KCF; ++q) a[m][h][q] = an[m][h][q];
      }
#pragma unroll
      for (int f = 0; f < FW; ++f) {
        const int cf = (wf * FW + f) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 4 * lk + v;  // f32 accumulator row within the 16x16 block
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
            const float e0 = acc[0][0][f][v], o0 = acc[0][1][f][v];
            const float y0 = e0 + o0, y0m = sig0 * (e0 - o0);
            const size_t p = INNER ? (size_t)col * N + i : (size_t)i * inner + col;
            const size_t pm = INNER ? (size_t)col * N + im : (size_t)im * inner + col;
            dst0[p] = G0 ? (float)(G0[i] * (double)y0) : y0;
            dst0[pm] = G0 ? (float)(G0[im] * (double)y0m) : y0m;
            if (NMAT > 1) {
              const float e1 = acc[NMAT - 1][0][f][v], o1 = acc[NMAT - 1][1][f][v];
              const float y1 = e1 + o1, y1m = sig1 * (e1 - o1);
              dst1[p] = (float)((G1 ? G1[i] * (double)y1 : (double)y1) + (G10 ? G10[i] * (double)y0 : 0.0));
              dst1[pm] = (float)((G1 ? G1[im] * (double)y1m : (double)y1m) + (G10 ? G10[im] * (double)y0m : 0.0));
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
// FP32 form of the copy-ahead pipelines of the folded contraction (the FP64
// ones are in contract.hip): a workgroup walks tpb tiles of one task; the
// next tile's raw input rows are copied into LDS (global_load_lds) while FP32
// MFMAs run on the current one; operator fragments stay in registers.  Each
// line is shifted by its middle-node value and folded in FP64, then cast.
// Strided axes (theta, phi): tiles of TC = 1024 / HP columns of N rows,
// inputs FP64 or FP32 per task; r axis: tiles of TL = 2048 / N whole lines,
// FP64 inputs.  Copy chunk q holds rows (lines) q, q + Q, ...; chunk pitches
// keep the fragment reads conflict-free (FP64 rows: 1152 bytes, FP32 rows:
// 1088, r lines: 1040).  Requirements (checked by the launcher): N = 2 HP,
// HP in {16, 32, 64}, whole tiles, row scales only on the r axis.
constexpr int P32_BUF = 16 * 1152;  // bytes per tile buffer (largest layout)

template <int HP, int NMAXT, bool INNER>
__global__ __launch_bounds__(256) void k_contract_f32_pipe(MixedTaskList tl, Bases B, const float* __restrict__ F0,
                                                           const float* __restrict__ F1,
                                                           const double* __restrict__ G0,
                                                           const double* __restrict__ G1,
                                                           const double* __restrict__ G10, float sig0, float sig1,
                                                           int inner, int slab, int ncb, int ntiles, int tpb,
                                                           long long P, JobSet js) {
  constexpr int N2 = 2 * HP;     // line length
  constexpr int NKS = HP / 4;    // k-steps of 4
  constexpr int TC = 1024 / HP;  // strided axes: columns per tile
  constexpr int TL = 2048 / N2;  // r axis: lines per tile
  constexpr int RT = HP / 16;    // 16-row output blocks
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const MixedTask tk = tl.t[blockIdx.z % tl.n];
  const long long jd = js.d[blockIdx.z / tl.n];
  F0 = shift_ptr(F0, jd);
  F1 = shift_ptr(F1, jd);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wa = wave % RT, wb = wave / RT;  // row block; column (strided) or line (r) block
  float* __restrict__ dst0 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst0 * (size_t)P;
  float* __restrict__ dst1 = (float*)shift_ptr(B.b[tk.dst_sel], jd) + (size_t)tk.dst1 * (size_t)P;
  const int t0 = blockIdx.x * tpb;
  const int nt = min(tpb, ntiles - t0);
  auto tile_off = [&](int t) -> size_t {
    const int g = t0 + t;
    if (INNER) return (size_t)g * TL * N2;
    const int sl = g / ncb, cb = g - sl * ncb;
    return (size_t)sl * (size_t)slab + (size_t)cb * TC;
  };

  auto body = [&](auto nm, auto es) {
    constexpr int NMAT = decltype(nm)::value;
    constexpr int ES = decltype(es)::value;  // input element bytes
    using T = typename std::conditional<ES == 8, double, float>::type;
    constexpr int CH = INNER ? 1040 : (ES == 8 ? 1152 : 1088);
    constexpr int RB = INNER ? ES * N2 : ES * TC;  // bytes per line (r) or row (strided)
    constexpr int LPR = RB / 16;                  // lanes per row in a copy
    constexpr int RPC = 64 / LPR;                 // rows per chunk
    constexpr int Q = (INNER ? TL : N2) / RPC;    // chunks per tile
    static_assert(Q % 4 == 0 && Q * CH <= P32_BUF, "chunk layout");
    const T* __restrict__ src = field_base<T>(tk, B, P, jd);
    const int cm = lane / LPR, cp = lane - cm * LPR;
    auto copy_tile = [&](int t, int b) {
      const T* g = src + tile_off(t) + (16 / ES) * cp;
      char* base = lds + b * P32_BUF;
#pragma unroll
      for (int q = wave; q < Q; q += 4)
        __builtin_amdgcn_global_load_lds((const void*)(g + (size_t)(q + Q * cm) * (INNER ? N2 : inner)),
                                         (lds_void_t*)(base + q * CH), 16, 0, 2);
    };
    // operator fragments: lane (lr, lk) holds E^T / O^T [4 ks + lk][16 wa + lr]
    const size_t hh = (size_t)HP * HP;
    float a[NMAT][2][NKS];
#pragma unroll
    for (int m = 0; m < NMAT; ++m) {
      const float* __restrict__ F = m == 0 ? F0 : F1;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) a[m][h][ks] = F[h * hh + (size_t)(4 * ks + lk) * HP + 16 * wa + lr];
    }
    // r axis: row scales of this lane's output rows i = 16 wa + lr and N - 1 - i
    const int ir = 16 * wa + lr, irm = N2 - 1 - ir;
    double s0 = 1.0, s0m = 1.0, s1 = 1.0, s1m = 1.0, s10 = 0.0, s10m = 0.0;
    if (INNER) {
      if (G0) { s0 = shift_ptr(G0, jd)[ir]; s0m = shift_ptr(G0, jd)[irm]; }
      if (G1) { s1 = shift_ptr(G1, jd)[ir]; s1m = shift_ptr(G1, jd)[irm]; }
      if (G10) { s10 = shift_ptr(G10, jd)[ir]; s10m = shift_ptr(G10, jd)[irm]; }
    }
    __builtin_amdgcn_s_waitcnt(0);  // fragments and scales in registers before the copies start
    copy_tile(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int own = 16 * wb + lr;  // strided: this lane's column; r: the line its fragment reads
    for (int t = 0; t < nt; ++t) {
      if (t > 0) {
        // tile t's copy was issued before the 8 NMAT stores of tile t - 1
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(8 * NMAT));
        lds_barrier();
      }
      if (t + 1 < nt) copy_tile(t + 1, (t + 1) & 1);
      const char* buf = lds + (t & 1) * P32_BUF;
      // the middle-node value of the line this lane's fragment reads
      const char* lp;
      const char* lm;
      double c;
      if (INNER) {
        lp = buf + (own % Q) * CH + (own / Q) * RB;
        lm = lp;
        c = (double)*(const T*)(lp + HP * ES);
      } else {
        lp = buf + lk * CH + own * ES;
        lm = buf - lk * CH + own * ES;
        c = (double)*(const T*)(buf + (HP % Q) * CH + (HP / Q) * RB + own * ES);
      }
      f4 acc[NMAT][2];
#pragma unroll
      for (int m = 0; m < NMAT; ++m) acc[m][0] = acc[m][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        double u, w;
        if (INNER) {
          const int k = 4 * ks + lk;
          u = (double)*(const T*)(lp + k * ES);
          w = (double)*(const T*)(lm + (N2 - 1 - k) * ES);
        } else {
          const int qa = (4 * ks) % Q, ma = (4 * ks) / Q;
          u = (double)*(const T*)(lp + qa * CH + ma * RB);
          w = (double)*(const T*)(lm + (Q - 1 - qa) * CH + (RPC - 1 - ma) * RB);
        }
        const double lo = u - c, hi = w - c;
        const float sk = (float)(lo + hi), dk = (float)(lo - hi);
#pragma unroll
        for (int m = 0; m < NMAT; ++m) {
          if (INNER) {
            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(sk, a[m][0][ks], acc[m][0], 0, 0, 0);
            acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(dk, a[m][1][ks], acc[m][1], 0, 0, 0);
          } else {
            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m][0][ks], sk, acc[m][0], 0, 0, 0);
            acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m][1][ks], dk, acc[m][1], 0, 0, 0);
          }
        }
      }
      // unfold, scale in FP64, store FP32: accumulator row 4 lk + v, column lr
      const size_t toff = tile_off(t);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        size_t p, pm;
        if (INNER) {  // rows: lines; columns: output rows ir
          const size_t l = toff + (size_t)(16 * wb + 4 * lk + v) * N2;
          p = l + ir;
          pm = l + irm;
        } else {  // rows: output rows i; columns: this lane's column
          const int i = 16 * wa + 4 * lk + v;
          p = toff + (size_t)i * inner + own;
          pm = toff + (size_t)(N2 - 1 - i) * inner + own;
        }
        const float e0 = acc[0][0][v], o0 = acc[0][1][v];
        const float y0 = e0 + o0, y0m = sig0 * (e0 - o0);
        dst0[p] = INNER ? (float)(s0 * (double)y0) : y0;
        dst0[pm] = INNER ? (float)(s0m * (double)y0m) : y0m;
        if (NMAT > 1) {
          const float e1 = acc[NMAT - 1][0][v], o1 = acc[NMAT - 1][1][v];
          const float y1 = e1 + o1, y1m = sig1 * (e1 - o1);
          dst1[p] = INNER ? (float)(s1 * (double)y1 + s10 * (double)y0) : y1;
          dst1[pm] = INNER ? (float)(s1m * (double)y1m + s10m * (double)y0m) : y1m;
        }
      }
    }
  };
  using I8 = std::integral_constant<int, 8>;
  using I4 = std::integral_constant<int, 4>;
  if (NMAXT > 1 && tk.nmat > 1) {
    using M = std::integral_constant<int, (NMAXT > 1 ? 2 : 1)>;
    if (!INNER && tk.src_f32) body(M{}, I4{});
    else body(M{}, I8{});
  } else {
    using M = std::integral_constant<int, 1>;
    if (!INNER && tk.src_f32) body(M{}, I4{});
    else body(M{}, I8{});
  }
}

template <int NMAT, bool INNER>
static hipError_t set_f32_fold_attr() {
  const int max_lds = 160 * 1024;
  const void* ks[] = {(const void*)k_contract_f32_fold<NMAT, INNER, 1>, (const void*)k_contract_f32_fold<NMAT, INNER, 2>,
                      (const void*)k_contract_f32_fold<NMAT, INNER, 4>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_contract_f32_fold(int axis, int nmat, const MixedTaskList& tl, const Bases& B,
                                    const FoldOp32& op0, const FoldOp32& op1, const double* g10, const int n[3],
                                    const int hpad[3], long long P, const JobSet& js, hipStream_t s) {
  if (tl.n <= 0) return hipSuccess;
  if (tl.n > MAX_TASKS || (nmat != 1 && nmat != 2) || axis < 0 || axis > 2 || js.n < 1 || js.n > MAXB)
    return hipErrorInvalidValue;
  const int N = n[axis], Hpad = hpad[axis];
  if ((N & 1) || Hpad < N / 2 || (Hpad & 15) || 2 * Hpad > 256) return hipErrorInvalidValue;
  int inner, outer, slab;
  geometry(axis, n, &inner, &outer, &slab);
  if ((Hpad == 16 || Hpad == 32 || Hpad == 64) && N == 2 * Hpad) {
    // copy-ahead pipeline: whole tiles, enough of them, FP64 inputs on the r
    // axis, row scales only there
    bool ok;
    int ntiles, ncb = 1;
    if (axis == 0) {
      const int tlines = 2048 / N;
      ok = inner % tlines == 0;
      for (int i = 0; i < tl.n && ok; ++i) ok = tl.t[i].src_f32 == 0;
      ntiles = inner / tlines;
    } else {
      const int tc = 1024 / Hpad;
      ok = inner % tc == 0 && op0.g == nullptr && op1.g == nullptr && g10 == nullptr;
      ncb = inner / tc;
      ntiles = ncb * outer;
    }
    // the kernel and its tiles per workgroup follow from one job's tiles, so
    // a job's arithmetic is the same alone and in a batch of any size
    const long long all = (long long)ntiles * tl.n;
    if (ok && all >= 2048) {
      const int tpb = (int)std::min(8LL, all / 1024);
      dim3 pg((ntiles + tpb - 1) / tpb, 1, tl.n * js.n);
#define LP(HPV, NM, IN)                                                                                          \
  hipLaunchKernelGGL((k_contract_f32_pipe<HPV, NM, IN>), pg, dim3(256), 2 * P32_BUF, s, tl, B, op0.et, op1.et, \
                     op0.g, op1.g, g10, (float)op0.sigma, (float)op1.sigma, inner, slab, ncb, ntiles, tpb, P, js)
#define LPA(HPV, IN)                     \
  do {                                   \
    if (nmat == 1) LP(HPV, 1, IN);       \
    else LP(HPV, 2, IN);                 \
  } while (0)
#define LPH(IN)                          \
  do {                                   \
    if (Hpad == 16) LPA(16, IN);         \
    else if (Hpad == 32) LPA(32, IN);    \
    else LPA(64, IN);                    \
  } while (0)
      if (axis == 0) LPH(true);
      else LPH(false);
#undef LPH
#undef LPA
#undef LP
      return hipGetLastError();
    }
  }
  dim3 grid((inner + MT_COLS - 1) / MT_COLS, outer, tl.n * js.n);
  const size_t lds = (size_t)2 * Hpad * F32_STRIDE * sizeof(float) + MT_COLS * sizeof(double);
  const int T = Hpad >> 4;
#define LF(NM, IN, W)                                                                                        \
  hipLaunchKernelGGL((k_contract_f32_fold<NM, IN, W>), grid, dim3(256), lds, s, tl, B, op0.et, op1.et, op0.g, \
                     op1.g, g10, (float)op0.sigma, (float)op1.sigma, N, Hpad, inner, slab, P, js)
#define LFW(NM, IN)                 \
  do {                              \
    if (T >= 4) LF(NM, IN, 4);      \
    else if (T >= 2) LF(NM, IN, 2); \
    else LF(NM, IN, 1);             \
  } while (0)
  if (axis == 0) {
    if (nmat == 1) LFW(1, true); else LFW(2, true);
  } else {
    if (nmat == 1) LFW(1, false); else LFW(2, false);
  }
#undef LFW
#undef LF
  return hipGetLastError();
}

template <int NMAT, bool INNER>
static hipError_t set_mixed_attr() {
  const int max_lds = 160 * 1024;
  const void* ks[] = {(const void*)k_contract_f32<NMAT, INNER, 1>, (const void*)k_contract_f32<NMAT, INNER, 2>,
                      (const void*)k_contract_f32<NMAT, INNER, 4>, (const void*)k_contract_bf3<NMAT, INNER, 1>,
                      (const void*)k_contract_bf3<NMAT, INNER, 2>, (const void*)k_contract_bf3<NMAT, INNER, 4>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t set_mixed_kernel_attributes() {
  hipError_t e = set_mixed_attr<1, true>();
  if (e == hipSuccess) e = set_mixed_attr<2, true>();
  if (e == hipSuccess) e = set_mixed_attr<1, false>();
  if (e == hipSuccess) e = set_mixed_attr<2, false>();
  if (e == hipSuccess) e = set_f32_fold_attr<1, true>();
  if (e == hipSuccess) e = set_f32_fold_attr<2, true>();
  if (e == hipSuccess) e = set_f32_fold_attr<1, false>();
  if (e == hipSuccess) e = set_f32_fold_attr<2, false>();
  return e;
}

hipError_t launch_contract_mixed(int prec, int axis, int nmat, const MixedTaskList& tl, const Bases& B,
                                 const MixedOps& op0, const MixedOps& op1, const int n[3],
                                 const int npad[3], long long P, const JobSet& js, hipStream_t s) {
  if (tl.n <= 0) return hipSuccess;
  if (tl.n > MAX_TASKS || (nmat != 1 && nmat != 2) || axis < 0 || axis > 2 || js.n < 1 || js.n > MAXB)
    return hipErrorInvalidValue;
  const int N = n[axis], Npad = npad[axis];
  int inner, outer, slab;
  geometry(axis, n, &inner, &outer, &slab);
  dim3 grid((inner + MT_COLS - 1) / MT_COLS, outer, tl.n * js.n);
  const size_t lds = mixed_lds_bytes(prec, Npad);
  const int T = Npad >> 4;
  if (prec == GRMHD_MIX_FP32) {
#define L32W(NM, IN, W)                                                                                  \
  hipLaunchKernelGGL((k_contract_f32<NM, IN, W>), grid, dim3(256), lds, s, tl, B, op0.f32, op1.f32, N, Npad, \
                     inner, slab, P, js)
#define L32(NM, IN)                        \
  do {                                      \
    if (T >= 4) L32W(NM, IN, 4);             \
    else if (T >= 2) L32W(NM, IN, 2);        \
    else L32W(NM, IN, 1);                    \
  } while (0)
    if (axis == 0) {
      if (nmat == 1) L32(1, true); else L32(2, true);
    } else {
      if (nmat == 1) L32(1, false); else L32(2, false);
    }
#undef L32
#undef L32W
  } else if (prec == GRMHD_MIX_BF16X3) {
    const int Kpad = round_up(Npad, 32);
#define LBFW(NM, IN, W)                                                                                  \
  hipLaunchKernelGGL((k_contract_bf3<NM, IN, W>), grid, dim3(256), lds, s, tl, B, op0.bhi, op0.blo, op1.bhi, \
                     op1.blo, N, Npad, Kpad, inner, slab, P, js)
#define LBF(NM, IN)                        \
  do {                                      \
    if (T >= 4) LBFW(NM, IN, 4);             \
    else if (T >= 2) LBFW(NM, IN, 2);        \
    else LBFW(NM, IN, 1);                    \
  } while (0)
    if (axis == 0) {
      if (nmat == 1) LBF(1, true); else LBF(2, true);
    } else {
      if (nmat == 1) LBF(1, false); else LBF(2, false);
    }
#undef LBF
#undef LBFW
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace grmhd
