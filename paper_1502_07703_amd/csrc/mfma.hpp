// Matrix-core (MFMA) building blocks for gfx950.
//
// All contractions of the hot path have the shape Y[i][j] = sum_k A[i][k] B[k][j]
// where the 16 rows i are (element, field) pairs of 4 elements x 4 fields,
// k runs over basis functions or cubature points, and j over cubature points,
// face points or basis functions.  With the 16x16x4 MFMA shapes, lane l of a
// wave holds (measured on gfx950 with one-hot operands)
//   A operand:  A[l % 16][l / 16]
//   B operand:  B[l / 16][l % 16]
//   D result, FP32 (v_mfma_f32_16x16x4f32):  D[4 (l / 16) + v][l % 16]
//   D result, FP64 (v_mfma_f64_16x16x4f64):  D[4 v + l / 16][l % 16],  v = 0..3.
// The row order of (element e, field f) is chosen per form so that in both
// cases lane l ends owning all four fields (register v = field) of element
// l / 16 at column l % 16 -- what the pointwise geometry and flux work needs:
// FP32 rows are i = 4 e + f, FP64 rows are i = 4 f + e.
// Operators are stored on the device in "fragment order", consecutive B
// operands interleaved by lane 16 bytes at a time (2 FP64 or 4 FP32
// fragments), so that one coalesced 16-byte-per-lane load fetches several
// operands: the vector-memory address unit, not bandwidth, limits a kernel
// that issues one narrow load per matrix-core product.
#pragma once

#include <hip/hip_runtime.h>

namespace dgpyr {

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

// 16-byte packs of operator fragments: KP fragments per lane per load.
typedef double dx2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Pack;
template <>
struct Pack<double> {
  using V = dx2;
  static constexpr int KP = 2;
};
template <>
struct Pack<float> {
  using V = fx4;
  static constexpr int KP = 4;
};

template <typename T>
__device__ __forceinline__ typename Pack<T>::V load_pack(const T* p) {
  return *reinterpret_cast<const typename Pack<T>::V*>(p);
}

// Precision forms of the contractions.  FORM 0: FP64 operands, FP64
// accumulation.  FORM 1: FP32 operands, FP32 accumulation.
template <int FORM>
struct Mma;

template <>
struct Mma<0> {
  using T = double;
  using Acc = dx4;
  static __device__ __forceinline__ int row(int e, int f) { return 4 * f + e; }
  static __device__ __forceinline__ int row_elem(int i) { return i & 3; }
  static __device__ __forceinline__ int row_field(int i) { return i >> 2; }
  static __device__ __forceinline__ Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mma<1> {
  using T = float;
  using Acc = fx4;
  static __device__ __forceinline__ int row(int e, int f) { return 4 * e + f; }
  static __device__ __forceinline__ int row_elem(int i) { return i >> 2; }
  static __device__ __forceinline__ int row_field(int i) { return i & 3; }
  static __device__ __forceinline__ Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Split-BF16 form: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a product
// is taken as hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x32_bf16 (FP32
// accumulation).  Lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7, and the result D[4 (l / 16) + v][l % 16]
// (measured on gfx950), so rows are i = 4 e + f as in the FP32 form.
typedef __bf16 bfx8 __attribute__((ext_vector_type(8)));

// The split is taken from x rounded to FP32 (the FP32 accumulation bounds
// the product's accuracy anyway): hi by round-to-nearest-even on the FP32
// bits, lo by the hardware conversion of the remainder xf - hi, which is exact
// in FP32.  About 6 vector instructions per value instead of 23 for the
// conversions from FP64; finite inputs only (a NaN does not survive the bit
// rounding; the FP64 state it came from keeps it).
__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float xf = (float)x;
  const uint32_t u = __float_as_uint(xf);
  const uint32_t hb = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  hi = __builtin_bit_cast(__bf16, (uint16_t)hb);
  lo = (__bf16)(xf - __uint_as_float(hb << 16));
}

__device__ __forceinline__ fx4 mma_bf16x3(bfx8 ah, bfx8 al, bfx8 bh, bfx8 bl, fx4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  return c;
}

// Tile counts for degree N.
template <int N>
struct Tiles {
  static constexpr int n1 = N + 1;
  static constexpr int Np = (N + 1) * (N + 2) * (2 * N + 3) / 6;
  static constexpr int Nc = n1 * n1 * n1;
  static constexpr int Nfq = n1 * n1;
  static constexpr int Nfc = 5 * Nfq;
  static constexpr int NCH = (Np + 3) / 4;     // k-chunks over basis functions
  static constexpr int NTC = (Nc + 15) / 16;   // 16-column tiles of volume points
  static constexpr int NTF = (Nfc + 15) / 16;  // 16-column tiles of face points
  static constexpr int NIT = (Np + 15) / 16;   // 16-column tiles of basis functions
  static constexpr int NCH32 = (Np + 31) / 32;  // 32-deep k-chunks over basis functions
  static constexpr int NT32C = (Nc + 31) / 32;  // 32-point chunks of volume points
  static constexpr int NT32F = (Nfc + 31) / 32; // 32-point chunks of face points
};

}  // namespace dgpyr
