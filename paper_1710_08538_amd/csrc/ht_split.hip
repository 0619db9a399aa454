// ht_split.hip -- emulated-FP64 matrix products on the low-precision matrix
// cores: the precision form of the WY updates.
//
// The paper runs every trailing update in FP64 (Sec. 3.3).  Here a product
// C = alpha op(A) op(B) + beta C with FP64 operands is formed from
// fixed-point digit slices instead (an error-free splitting in the spirit of
// Ozaki et al., 2012):
//
//   For every K-chunk of SKC contraction indices, each row of op(A) gets a
//   power-of-two exponent e (its largest magnitude in the chunk lies below
//   2^e), and the row is written as
//       a = 2^e * ( sum_{i < ns} d_i 2^{-b (i+1)} + rho ),  |rho| < 2^{-b ns},
//   with integer digits |d_i| <= 2^b - 1 (truncated expansion, so every digit
//   and the remainder are exact in FP64).  Columns of op(B) get the same
//   treatment.  Digit width b = 7 (BF16: integers up to 256 are exact) or
//   b = 4 (FP8 E4M3: integers up to 16 are exact).
//
//   The product of slice i of A and slice j of B carries the weight
//   2^{-b (i+j+2)}.  Slice pairs of one level L = i + j (L < ns) share one
//   FP32 accumulator: each digit product is below 2^{2b}, so a level's sum
//   over the chunk is an integer below ns * SKC * 2^{2b} <= 2^24 and the
//   MFMA accumulation is exact.  The levels are then combined in FP64 with
//   their weights and scaled by 2^{e_row + e_col}; chunks add up in FP64.
//
//   Dropped terms bound the error of one product per contraction index:
//   the slice pairs of levels >= ns contribute less than (ns + 2.1)
//   2^{-b ns} and the remainders less than 2^{1 - b ns}, both times
//   2^{e_row + e_col}.
//
// One 256-thread workgroup computes a 64 x 64 tile of C; each wavefront owns
// a 32 x 32 quarter (2 x 2 MFMA blocks of 16 x 16).  Per chunk the
// workgroup loads the 64 x SKC slab of op(A) and SKC x 64 slab of op(B),
// splits them into digit slices in LDS (four threads per row / column,
// eight entries each, the exponent from a four-lane max), then runs the
// levels' MFMAs from LDS.
//
// MFMA operand layouts (lane l of the wavefront), one instruction per
// 32-digit chunk in both formats:
//   v_mfma_f32_16x16x32_bf16:  A[l%16][8(l/16) + 0..7],  B[8(l/16) + 0..7][l%16]
//   v_mfma_f32_16x16x32_fp8:   A[l%16][8(l/16) + 0..7],  B[8(l/16) + 0..7][l%16]
//   result register q:         C[4(l/16) + q][l%16]
#include "ht_device.h"
#include "ht_internal.h"

namespace htk {

namespace {

constexpr int SBM = 64;   // tile rows
constexpr int SBN = 64;   // tile columns
constexpr int SKC = 32;   // contraction chunk

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Digit formats.  RS: bytes per LDS row of one slice (SKC digits + padding,
// a multiple of 8 so every fragment is read with aligned 8-byte loads; two
// of them for the 16 bytes of eight BF16 digits).  Frag: one lane's operand.
template <int FMT>
struct Fmt;
template <>
struct Fmt<0> {  // BF16 digits, 7 bits + sign
  static constexpr int bits = 7;
  static constexpr int kstep = 32;
  static constexpr int RS = (SKC + 4) * 2;
  typedef uint4 Frag;
};
template <>
struct Fmt<1> {  // FP8 E4M3 digits, 4 bits + sign
  static constexpr int bits = 4;
  static constexpr int kstep = 32;
  static constexpr int RS = SKC + 8;
  typedef uint2 Frag;
};

constexpr int kSliceBytes = 36864;  // per operand: 8 BF16 slices or 14 FP8 slices

struct SplitArgs {
  int m, n, k, ns;
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  int lda, ldb, ldc;
};

// Eight digits of one slice, packed as they are stored in LDS.
template <int FMT>
__device__ __forceinline__ uint2 pack_digits(const double (&d)[8]);

template <>
__device__ __forceinline__ uint2 pack_digits<0>(const double (&d)[8]) {
  // |d| <= 127: the float is exact and its upper 16 bits are the BF16 value
  uint32_t h[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) h[u] = __float_as_uint((float)d[u]) >> 16;
  // only the first four digits fit in 8 bytes; the caller stores two halves
  return make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

__device__ __forceinline__ uint2 pack_bf16_hi(const double (&d)[8]) {
  uint32_t h[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) h[u] = __float_as_uint((float)d[4 + u]) >> 16;
  return make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

template <>
__device__ __forceinline__ uint2 pack_digits<1>(const double (&d)[8]) {
  // |d| <= 15: exact in E4M3 (the hardware conversion picks the encoding)
  int w0 = __builtin_amdgcn_cvt_pk_fp8_f32((float)d[0], (float)d[1], 0, false);
  w0 = __builtin_amdgcn_cvt_pk_fp8_f32((float)d[2], (float)d[3], w0, true);
  int w1 = __builtin_amdgcn_cvt_pk_fp8_f32((float)d[4], (float)d[5], 0, false);
  w1 = __builtin_amdgcn_cvt_pk_fp8_f32((float)d[6], (float)d[7], w1, true);
  return make_uint2((uint32_t)w0, (uint32_t)w1);
}

// Split eight entries x (one row of a chunk, its four-lane group holding the
// rest of the row) into ns digit slices at dst + i * 64 * RS; returns the
// exponent e of the row (2^e above its largest magnitude, 0 for a zero row).
template <int FMT>
__device__ __forceinline__ int split_row(double (&x)[8], int ns, unsigned char* dst) {
  constexpr int RS = Fmt<FMT>::RS;
  double amx = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) amx = fmax(amx, fabs(x[u]));
  amx = fmax(amx, __shfl_xor(amx, 1, 64));
  amx = fmax(amx, __shfl_xor(amx, 2, 64));
  const int e = (amx > 0.0) ? ilogb(amx) + 1 : 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) x[u] = ldexp(x[u], -e);
  const double scale = (double)(1 << Fmt<FMT>::bits);
  for (int i = 0; i < ns; ++i) {
    double d[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[u] *= scale;       // exact: a power of two
      d[u] = trunc(x[u]);  // |d| <= 2^b - 1
      x[u] -= d[u];        // exact: the fractional part
    }
    unsigned char* p = dst + (size_t)i * 64 * RS;
    if (FMT == 0) {
      *(uint2*)p = pack_digits<0>(d);
      *(uint2*)(p + 8) = pack_bf16_hi(d);
    } else {
      *(uint2*)p = pack_digits<1>(d);
    }
  }
  return e;
}

// One lane's operand from a slice row (8-byte aligned).
template <int FMT>
__device__ __forceinline__ typename Fmt<FMT>::Frag load_frag(const unsigned char* p);
template <>
__device__ __forceinline__ uint4 load_frag<0>(const unsigned char* p) {
  const uint2 lo = *(const uint2*)p, hi = *(const uint2*)(p + 8);
  return make_uint4(lo.x, lo.y, hi.x, hi.y);
}
template <>
__device__ __forceinline__ uint2 load_frag<1>(const unsigned char* p) {
  return *(const uint2*)p;
}

template <int FMT>
__device__ __forceinline__ v4f mfma_digits(typename Fmt<FMT>::Frag a, typename Fmt<FMT>::Frag b, v4f c);

template <>
__device__ __forceinline__ v4f mfma_digits<0>(uint4 a, uint4 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v4f mfma_digits<1>(uint2 a, uint2 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                    __builtin_bit_cast(long, b), c, 0, 0, 0);
}

template <int FMT, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_split_gemm(SplitArgs a) {
  constexpr int RS = Fmt<FMT>::RS;
  constexpr int KSTEP = Fmt<FMT>::kstep;
  constexpr int NKS = SKC / KSTEP;
  __shared__ __align__(16) unsigned char AD[kSliceBytes];
  __shared__ __align__(16) unsigned char BD[kSliceBytes];
  __shared__ int ea[SBM], eb[SBN];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r0 = blockIdx.x * SBM, c0 = blockIdx.y * SBN;
  const int ns = a.ns;
  const int lr = tid >> 2, q4 = tid & 3;
  // MFMA role: wavefront quarter (wr, wc), lane row/column within a block
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;
  const int fr = lane & 15, fk = (lane >> 4) * (KSTEP / 4);

  double c64[2][2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) c64[rb][cb][q] = 0.0;

  // loader role: row r0+lr of op(A) and column c0+lr of op(B), entries
  // 8 q4 .. 8 q4 + 7 of a chunk; the next chunk's entries are loaded while
  // the current chunk's MFMAs run
  const int gr = r0 + lr, gc = c0 + lr;
  double xa[8], xb[8];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kk = k0 + 8 * q4 + u;
      xa[u] = (gr < a.m && kk < a.k)
                  ? (TA ? a.A[(size_t)kk + (size_t)gr * a.lda] : a.A[(size_t)gr + (size_t)kk * a.lda])
                  : 0.0;
      xb[u] = (gc < a.n && kk < a.k)
                  ? (TB ? a.B[(size_t)gc + (size_t)kk * a.ldb] : a.B[(size_t)kk + (size_t)gc * a.ldb])
                  : 0.0;
    }
  };
  load_chunk(0);
  for (int k0 = 0; k0 < a.k; k0 += SKC) {
    // ---- split the chunk of op(A) and op(B) into LDS, then fetch the next
    {
      const int e = split_row<FMT>(xa, ns, AD + lr * RS + 8 * q4 * (FMT == 0 ? 2 : 1));
      if (q4 == 0) ea[lr] = e;
    }
    {
      const int e = split_row<FMT>(xb, ns, BD + lr * RS + 8 * q4 * (FMT == 0 ? 2 : 1));
      if (q4 == 0) eb[lr] = e;
    }
    if (k0 + SKC < a.k) load_chunk(k0 + SKC);
    __syncthreads();

    // ---- levels: sum over slice pairs (i, L - i), weight 2^{-b (L + 2)}
    double tacc[2][2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) tacc[rb][cb][q] = 0.0;
    for (int L = 0; L < ns; ++L) {
      v4f acc[2][2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
      for (int i = 0; i <= L; ++i) {
        const unsigned char* As = AD + (size_t)i * 64 * RS;
        const unsigned char* Bs = BD + (size_t)(L - i) * 64 * RS;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          const int kb = (ks * KSTEP + fk) * (FMT == 0 ? 2 : 1);
          typedef typename Fmt<FMT>::Frag Frag;
          Frag af[2], bf[2];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) af[rb] = load_frag<FMT>(As + (wr + 16 * rb + fr) * RS + kb);
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) bf[cb] = load_frag<FMT>(Bs + (wc + 16 * cb + fr) * RS + kb);
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mfma_digits<FMT>(af[rb], bf[cb], acc[rb][cb]);
        }
      }
      const double w = ldexp(1.0, -Fmt<FMT>::bits * (L + 2));
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int q = 0; q < 4; ++q) tacc[rb][cb][q] = fma((double)acc[rb][cb][q], w, tacc[rb][cb][q]);
    }
    // ---- scale by the row and column exponents of this chunk
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = wr + 16 * rb + 4 * (lane >> 4) + q, cc = wc + 16 * cb + fr;
          c64[rb][cb][q] += ldexp(tacc[rb][cb][q], ea[rr] + eb[cc]);
        }
    __syncthreads();  // slices and exponents are rewritten by the next chunk
  }

#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = r0 + wr + 16 * rb + 4 * (lane >> 4) + q, gc = c0 + wc + 16 * cb + fr;
        if (gr < a.m && gc < a.n) {
          double* p = a.C + (size_t)gr + (size_t)gc * a.ldc;
          *p = (a.beta == 0.0) ? a.alpha * c64[rb][cb][q] : fma(a.alpha, c64[rb][cb][q], a.beta * *p);
        }
      }
}

template <int FMT>
void launch_split(hipStream_t st, bool ta, bool tb, dim3 grid, const SplitArgs& sa) {
  if (!ta && !tb) hipLaunchKernelGGL((k_split_gemm<FMT, false, false>), grid, dim3(256), 0, st, sa);
  else if (ta && !tb) hipLaunchKernelGGL((k_split_gemm<FMT, true, false>), grid, dim3(256), 0, st, sa);
  else if (!ta && tb) hipLaunchKernelGGL((k_split_gemm<FMT, false, true>), grid, dim3(256), 0, st, sa);
  else hipLaunchKernelGGL((k_split_gemm<FMT, true, true>), grid, dim3(256), 0, st, sa);
}

}  // namespace

int split_max_slices(int fmt) { return fmt == 0 ? 8 : 14; }
int split_default_slices(int fmt) { return fmt == 0 ? 8 : 14; }

void split_gemm(hipStream_t st, int fmt, int ns, bool transA, bool transB, int m, int n, int k,
                double alpha, const double* A, int lda, const double* B, int ldb, double beta,
                double* C, int ldc) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0) {  // C = beta C: the FP64 path handles the scaling
    gemm(st, transA, transB, m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc);
    return;
  }
  SplitArgs sa;
  sa.m = m;
  sa.n = n;
  sa.k = k;
  sa.ns = ns;
  sa.alpha = alpha;
  sa.beta = beta;
  sa.A = A;
  sa.B = B;
  sa.C = C;
  sa.lda = lda;
  sa.ldb = ldb;
  sa.ldc = ldc;
  dim3 grid((m + SBM - 1) / SBM, (n + SBN - 1) / SBN);
  if (fmt == 0) launch_split<0>(st, transA, transB, grid, sa);
  else launch_split<1>(st, transA, transB, grid, sa);
}

}  // namespace htk
