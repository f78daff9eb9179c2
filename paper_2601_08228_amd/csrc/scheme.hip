// Lifting with chosen predict and update operators along mode 3 (Sec. II-A,
// W_j built from P_j and U_j; Remark 3.1), its inverse and both transposes,
// for gfx950.
//
// Per level j the current smooth sequence of a tube splits into pairs; o[m]
// is the first entry of pair m and e[m] the second.  The forward level is
// d = o - P e, s = e + U d, with P and U 5-tap stencils (offsets -2..2,
// indices clamped to the ends of the level's sequence); P = I, U = I/2 is the
// lazy transform.
//
// With stencils a level couples neighbouring pairs, so unlike the lazy pass a
// tube cannot be cut into independent blocks of 2^L slices.  A workgroup owns
// a tile of TP neighbouring positions (TP whole tubes): it reads the p x TP
// tile into LDS once (each slice contributes TP consecutive elements, a
// coalesced stream), runs every level in LDS and writes the p x TP result
// once, so each tensor still crosses HBM once per pass.
//
// In-place layout in LDS: the level-(j-1) smooth sequence sits in rows
// (h - 1) + k h, h = 2^(j-1).  Pair m of level j has o in row h - 1 + 2 m h
// and e in row h - 1 + (2 m + 1) h; d overwrites o and s overwrites e, so
// s_j lands in rows (2h - 1) + m 2h, the layout of level j + 1.  A level is
// two half-steps, each reading one set of rows and writing the other, with a
// barrier between them.  Transposed stencils are gathers: (S^T g)[i] sums
// tap_t g[m] over the m, t with clamp(m + t - 2) = i.

#include "wp_internal.h"

namespace wp {
namespace {

constexpr int kSchemeThreads = 256;

// Row of Mallat coefficient c (s_L first, then d_L, ..., d_1) in the in-place
// layout.
__device__ __forceinline__ int coeff_row(int c, int p, int L) {
  if (c < (p >> L)) return ((1 << L) - 1) + (c << L);
  int j = L;
  while (c >= (p >> (j - 1))) --j;  // d_j occupies [p >> j, p >> (j - 1))
  const int m = c - (p >> j);
  return ((1 << (j - 1)) - 1) + (m << j);
}

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// V consecutive positions as one vector (16-byte loads and LDS accesses when
// V * sizeof(T) = 16).
template <typename T, int V>
using Vec = T __attribute__((ext_vector_type(V)));

// sum_t w[t] g[clamp(m + t - 2)] over rows g(k) = buf[base + k * stride] (a
// row is TP / V vectors wide; `col` selects this thread's vector).
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> stencil(const Vec<T, V>* buf, const double* w, int m, int n,
                                             int base, int stride, int rowv, int col) {
  Vec<T, V> acc = T(0);
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    if (w[t] == 0.0) continue;
    const int k = clampi(m + t - 2, n - 1);
    acc += T(w[t]) * buf[(base + k * stride) * rowv + col];
  }
  return acc;
}

// Transposed stencil: sum over m, t with clamp(m + t - 2) = i of w[t] g(m).
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> stencil_t(const Vec<T, V>* buf, const double* w, int i,
                                               int n, int base, int stride, int rowv, int col) {
  Vec<T, V> acc = T(0);
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    if (w[t] == 0.0) continue;
    const int off = t - 2;
    int lo, hi;
    if (n == 1) {
      lo = 0;
      hi = 0;
    } else if (i == 0) {  // m + off <= 0
      lo = 0;
      hi = -off < n - 1 ? -off : n - 1;
    } else if (i == n - 1) {  // m + off >= n - 1
      lo = n - 1 - off > 0 ? n - 1 - off : 0;
      hi = n - 1;
    } else {
      lo = hi = i - off;
      if (lo < 0 || lo > n - 1) continue;
    }
    for (int m = lo; m <= hi; ++m) acc += T(w[t]) * buf[(base + m * stride) * rowv + col];
  }
  return acc;
}

// Rows per batch of global loads (kept in registers before the LDS stores,
// so that a thread has that many loads in flight).
constexpr int kBatch = 8;

template <typename T, int V, LiftKind K, bool SPLIT>
__global__ __launch_bounds__(kSchemeThreads) void lift_scheme_kernel(
    const T* __restrict__ in, T* __restrict__ out, uint16_t* __restrict__ hi,
    uint16_t* __restrict__ lo, int64_t P, int p, int L, int tp, SchemeTaps taps) {
  using VT = Vec<T, V>;
  extern __shared__ unsigned char s_raw[];
  VT* buf = reinterpret_cast<VT*>(s_raw);
  const int rowv = tp / V;                   // vectors per row
  const int col = threadIdx.x % rowv;
  const int r0 = threadIdx.x / rowv;
  const int rstep = kSchemeThreads / rowv;
  const int64_t pos = int64_t(blockIdx.x) * tp + int64_t(col) * V;
  const bool live = pos < P;                 // P is a multiple of V
  constexpr bool kCoeffIn = K == LiftKind::kInverse || K == LiftKind::kForwardAdj;

  for (int c0 = r0; c0 < p; c0 += rstep * kBatch) {
    VT v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = c0 + u * rstep;
      v[u] = (live && c < p) ? *reinterpret_cast<const VT*>(in + int64_t(c) * P + pos) : VT(T(0));
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = c0 + u * rstep;
      if (c < p) buf[(kCoeffIn ? coeff_row(c, p, L) : c) * rowv + col] = v[u];
    }
  }
  __syncthreads();

  if constexpr (K == LiftKind::kForward || K == LiftKind::kInverseAdj) {
    for (int j = 1; j <= L; ++j) {
      const int h = 1 << (j - 1), n = p >> j;
      const int ob = h - 1, eb = 2 * h - 1, st = 2 * h;  // o rows ob + m st, e rows eb + m st
      const double* pw = taps.w[j - 1][0];
      const double* uw = taps.w[j - 1][1];
      if constexpr (K == LiftKind::kForward) {
        for (int m = r0; m < n; m += rstep)  // d = o - P e
          buf[(ob + m * st) * rowv + col] -= stencil<T, V>(buf, pw, m, n, eb, st, rowv, col);
        __syncthreads();
        for (int m = r0; m < n; m += rstep)  // s = e + U d
          buf[(eb + m * st) * rowv + col] += stencil<T, V>(buf, uw, m, n, ob, st, rowv, col);
      } else {
        for (int i = r0; i < n; i += rstep)  // g_s = g_e + P^T g_o
          buf[(eb + i * st) * rowv + col] += stencil_t<T, V>(buf, pw, i, n, ob, st, rowv, col);
        __syncthreads();
        for (int i = r0; i < n; i += rstep)  // g_d = g_o - U^T g_s
          buf[(ob + i * st) * rowv + col] -= stencil_t<T, V>(buf, uw, i, n, eb, st, rowv, col);
      }
      __syncthreads();
    }
  } else {
    for (int j = L; j >= 1; --j) {
      const int h = 1 << (j - 1), n = p >> j;
      const int ob = h - 1, eb = 2 * h - 1, st = 2 * h;
      const double* pw = taps.w[j - 1][0];
      const double* uw = taps.w[j - 1][1];
      if constexpr (K == LiftKind::kInverse) {
        for (int m = r0; m < n; m += rstep)  // e = s - U d
          buf[(eb + m * st) * rowv + col] -= stencil<T, V>(buf, uw, m, n, ob, st, rowv, col);
        __syncthreads();
        for (int m = r0; m < n; m += rstep)  // o = d + P e
          buf[(ob + m * st) * rowv + col] += stencil<T, V>(buf, pw, m, n, eb, st, rowv, col);
      } else {
        for (int i = r0; i < n; i += rstep)  // g_o = g_d + U^T g_s
          buf[(ob + i * st) * rowv + col] += stencil_t<T, V>(buf, uw, i, n, eb, st, rowv, col);
        __syncthreads();
        for (int i = r0; i < n; i += rstep)  // g_e = g_s - P^T g_o
          buf[(eb + i * st) * rowv + col] -= stencil_t<T, V>(buf, pw, i, n, ob, st, rowv, col);
      }
      __syncthreads();
    }
  }

  if (!live) return;
  for (int c = r0; c < p; c += rstep) {
    const VT v = buf[(kCoeffIn ? c : coeff_row(c, p, L)) * rowv + col];
    if constexpr (SPLIT) {
      // bf16 hi and the bf16 residual, both rounded to nearest even; x - hi is
      // exact in FP32.
      using HV = Vec<uint16_t, V>;
      HV h, l;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const __bf16 hb = static_cast<__bf16>(v[i]);
        h[i] = __builtin_bit_cast(uint16_t, hb);
        l[i] = __builtin_bit_cast(uint16_t,
                                  static_cast<__bf16>(float(v[i]) - static_cast<float>(hb)));
      }
      *reinterpret_cast<HV*>(hi + int64_t(c) * P + pos) = h;
      if (lo != nullptr) *reinterpret_cast<HV*>(lo + int64_t(c) * P + pos) = l;
    } else {
      *reinterpret_cast<VT*>(out + int64_t(c) * P + pos) = v;
    }
  }
}

template <typename T, int V, LiftKind K, bool SPLIT>
hipError_t launch_v(const T* in, T* out, uint16_t* hi, uint16_t* lo, int64_t P, int64_t p,
                    int L, const SchemeTaps& taps, hipStream_t s) {
  int tp = scheme_tile_positions(p, sizeof(T));
  if (tp == 0) return hipErrorInvalidValue;
  while (tp > V && int64_t(tp / 2) >= P) tp /= 2;  // no wider than the tensor
  const size_t lds = size_t(p) * tp * sizeof(T);
  auto kern = lift_scheme_kernel<T, V, K, SPLIT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  const int64_t grid = (P + tp - 1) / tp;
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(kSchemeThreads), lds, s, in, out, hi, lo, P,
                     int(p), L, tp, taps);
  return hipGetLastError();
}

inline bool aligned16(const void* x) { return (reinterpret_cast<uintptr_t>(x) & 15) == 0; }

// 16-byte vectors when every row of the tensor starts on a 16-byte boundary.
template <typename T, LiftKind K, bool SPLIT>
hipError_t launch_one(const T* in, T* out, uint16_t* hi, uint16_t* lo, int64_t P, int64_t p,
                      int L, const SchemeTaps& taps, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  const bool vec = P % V == 0 && aligned16(in) && (SPLIT ? (P % 8 == 0 && aligned16(hi) &&
                                                            (lo == nullptr || aligned16(lo)))
                                                         : aligned16(out));
  if (vec) return launch_v<T, V, K, SPLIT>(in, out, hi, lo, P, p, L, taps, s);
  return launch_v<T, 1, K, SPLIT>(in, out, hi, lo, P, p, L, taps, s);
}

template <typename T>
hipError_t dispatch(LiftKind kind, const T* in, T* out, int64_t P, int64_t p, int L,
                    const SchemeTaps& taps, hipStream_t s) {
  switch (kind) {
    case LiftKind::kForward:
      return launch_one<T, LiftKind::kForward, false>(in, out, nullptr, nullptr, P, p, L, taps, s);
    case LiftKind::kInverse:
      return launch_one<T, LiftKind::kInverse, false>(in, out, nullptr, nullptr, P, p, L, taps, s);
    case LiftKind::kForwardAdj:
      return launch_one<T, LiftKind::kForwardAdj, false>(in, out, nullptr, nullptr, P, p, L, taps,
                                                         s);
    case LiftKind::kInverseAdj:
      return launch_one<T, LiftKind::kInverseAdj, false>(in, out, nullptr, nullptr, P, p, L, taps,
                                                         s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int scheme_tile_positions(int64_t p, size_t es) {
  // Widest power-of-two tile (up to 256 positions) within 32 KiB of LDS, at
  // least 16 positions; 0 if 16 positions would need more than 128 KiB.
  int tp = 256;
  while (tp > 16 && size_t(p) * tp * es > 32768) tp /= 2;
  return size_t(p) * tp * es <= 131072 ? tp : 0;
}

hipError_t launch_lift_scheme_f64(LiftKind kind, const double* in, double* out, int64_t P,
                                  int64_t p, int L, const SchemeTaps& taps, hipStream_t s) {
  return dispatch<double>(kind, in, out, P, p, L, taps, s);
}

hipError_t launch_lift_scheme_f32(LiftKind kind, const float* in, float* out, int64_t P,
                                  int64_t p, int L, const SchemeTaps& taps, hipStream_t s) {
  return dispatch<float>(kind, in, out, P, p, L, taps, s);
}

hipError_t launch_lift_scheme_f32_split(LiftKind kind, const float* in, uint16_t* hi,
                                        uint16_t* lo, int64_t P, int64_t p, int L,
                                        const SchemeTaps& taps, hipStream_t s) {
  if (kind == LiftKind::kForward)
    return launch_one<float, LiftKind::kForward, true>(in, nullptr, hi, lo, P, p, L, taps, s);
  if (kind == LiftKind::kInverseAdj)
    return launch_one<float, LiftKind::kInverseAdj, true>(in, nullptr, hi, lo, P, p, L, taps, s);
  return hipErrorInvalidValue;  // split output is for coefficient-producing passes
}

}  // namespace wp
