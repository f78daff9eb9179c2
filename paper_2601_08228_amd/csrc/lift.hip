// Lazy lifting passes along mode 3 (Sec. II-A, Eq. (1), Alg. 1 outer steps)
// and their transposes, for gfx950.
//
// Every thread owns V consecutive elements of a frontal slice (one position
// of V neighbouring mode-3 tubes) and one block of 2^L consecutive slices.
// With P_j = I and U_j = I/2 the level-j support is a disjoint block of 2^j
// slices, so a block of 2^L slices is transformed with no halo and no
// communication: the thread loads the whole block, runs every level in
// registers and stores every coefficient once.  A wavefront reads and writes
// 64*V consecutive elements of one slice per access, so every HBM access is
// a coalesced 256 B..1 KiB stream and each tensor crosses HBM exactly once
// per pass (read once, written once).
//
// Up to 10 levels are handled with two register tiers: the inner tier runs
// levels 1..LI on sub-blocks of 2^LI slices, one sub-block at a time, and
// keeps each sub-block's smooth value; the outer tier runs levels LI+1..L on
// those 2^LO values.

#include "wp_internal.h"

namespace wp {
namespace {

constexpr int kThreads = 256;

// ---- per-level arithmetic --------------------------------------------------
// Analysis passes map a pair (first, second) to (smooth, detail); synthesis
// passes map (smooth, detail) back to (first, second).  The operation order
// is the one of the level steps (d/2 is an exact scaling), so the FP64 pass
// rounds exactly like a literal evaluation of those steps.
template <LiftKind K>
struct Level;

template <>
struct Level<LiftKind::kForward> {  // d = first - second, s = second + d/2
  static constexpr bool kAnalysis = true;
  template <typename T>
  __device__ static void op(T a, T b, T& s, T& d) {
    d = a - b;
    s = b + d * T(0.5);
  }
};

template <>
struct Level<LiftKind::kInverseAdj> {  // transpose of one inverse level
  static constexpr bool kAnalysis = true;
  template <typename T>
  __device__ static void op(T a, T b, T& s, T& d) {
    s = a + b;
    d = (a - b) * T(0.5);
  }
};

template <>
struct Level<LiftKind::kInverse> {  // second = s - d/2, first = d + second
  static constexpr bool kAnalysis = false;
  template <typename T>
  __device__ static void op(T s, T d, T& a, T& b) {
    b = s - d * T(0.5);
    a = d + b;
  }
};

template <>
struct Level<LiftKind::kForwardAdj> {  // transpose of one forward level
  static constexpr bool kAnalysis = false;
  template <typename T>
  __device__ static void op(T s, T d, T& a, T& b) {
    a = s * T(0.5) + d;
    b = s * T(0.5) - d;
  }
};

// ---- vector access ---------------------------------------------------------
template <typename T, int V>
struct Pack {
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack(const T* __restrict__ p) {
  Pack<T, V> r;
  if constexpr (sizeof(T) * V == 16) {
    using U = unsigned int __attribute__((ext_vector_type(4)));
    U x = *reinterpret_cast<const U*>(p);
    __builtin_memcpy(&r, &x, 16);
  } else if constexpr (sizeof(T) * V == 8) {
    using U = unsigned int __attribute__((ext_vector_type(2)));
    U x = *reinterpret_cast<const U*>(p);
    __builtin_memcpy(&r, &x, 8);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = p[i];
  }
  return r;
}

template <typename T, int V>
__device__ __forceinline__ void store_pack(T* __restrict__ p, const Pack<T, V>& r) {
  if constexpr (sizeof(T) * V == 16) {
    using U = unsigned int __attribute__((ext_vector_type(4)));
    U x;
    __builtin_memcpy(&x, &r, 16);
    *reinterpret_cast<U*>(p) = x;
  } else if constexpr (sizeof(T) * V == 8) {
    using U = unsigned int __attribute__((ext_vector_type(2)));
    U x;
    __builtin_memcpy(&x, &r, 8);
    *reinterpret_cast<U*>(p) = x;
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) p[i] = r.v[i];
  }
}

// ---- coefficient stores ----------------------------------------------------
template <typename T, int V>
struct PlainStore {
  T* __restrict__ out;
  int64_t P;
  __device__ __forceinline__ void put(int64_t slice, int64_t off, const Pack<T, V>& x) const {
    store_pack<T, V>(out + slice * P + off, x);
  }
};

template <int V>
struct SplitStore {
  uint16_t* __restrict__ hi;
  uint16_t* __restrict__ lo;  // may be null
  int64_t P;
  __device__ __forceinline__ void put(int64_t slice, int64_t off, const Pack<float, V>& x) const {
    // bf16 conversions round to nearest even (v_cvt_pk_bf16_f32); x - hi is
    // exact in FP32, so lo is the correctly rounded residual.
    Pack<uint16_t, V> h, l;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const __bf16 hb = static_cast<__bf16>(x.v[i]);
      const __bf16 lb = static_cast<__bf16>(x.v[i] - static_cast<float>(hb));
      h.v[i] = __builtin_bit_cast(uint16_t, hb);
      l.v[i] = __builtin_bit_cast(uint16_t, lb);
    }
    store_pack<uint16_t, V>(hi + slice * P + off, h);
    if (lo != nullptr) store_pack<uint16_t, V>(lo + slice * P + off, l);
  }
};

template <typename T, int V, class Op>
__device__ __forceinline__ void apply_pair(const Pack<T, V>& x, const Pack<T, V>& y, Pack<T, V>& u,
                                           Pack<T, V>& w) {
#pragma unroll
  for (int i = 0; i < V; ++i) Op::op(x.v[i], y.v[i], u.v[i], w.v[i]);
}

// ---- analysis pass: spatial block -> Eq. (1)-ordered coefficients ----------
template <typename T, int V, int LI, int LO, LiftKind K, class Store>
__global__ __launch_bounds__(kThreads) void lift_analysis(const T* __restrict__ in, Store st,
                                                          int64_t P, int64_t p, int64_t nvec,
                                                          int64_t nblk_pos) {
  using Op = Level<K>;
  constexpr int L = LI + LO;
  constexpr int NI = 1 << LI;
  constexpr int NO = 1 << LO;
  const int64_t b = blockIdx.x / nblk_pos;
  const int64_t e = (blockIdx.x % nblk_pos) * kThreads + threadIdx.x;
  if (e >= nvec) return;
  const int64_t off = e * V;

  Pack<T, V> S[NO];
#pragma unroll
  for (int sb = 0; sb < NO; ++sb) {
    Pack<T, V> v[NI];
    const int64_t base = b * (NI * NO) + sb * NI;
#pragma unroll
    for (int t = 0; t < NI; ++t) v[t] = load_pack<T, V>(in + (base + t) * P + off);
#pragma unroll
    for (int j = 1; j <= LI; ++j) {
      const int half = NI >> j;
      const int64_t dbase = (p >> j) + b * (int64_t(1) << (L - j)) + int64_t(sb) * half;
#pragma unroll
      for (int q = 0; q < half; ++q) {
        Pack<T, V> s, d;
        apply_pair<T, V, Op>(v[2 * q], v[2 * q + 1], s, d);
        st.put(dbase + q, off, d);
        v[q] = s;
      }
    }
    S[sb] = v[0];
  }
#pragma unroll
  for (int jo = 1; jo <= LO; ++jo) {
    const int j = LI + jo;
    const int half = NO >> jo;
    const int64_t dbase = (p >> j) + b * (int64_t(1) << (L - j));
#pragma unroll
    for (int q = 0; q < half; ++q) {
      Pack<T, V> s, d;
      apply_pair<T, V, Op>(S[2 * q], S[2 * q + 1], s, d);
      st.put(dbase + q, off, d);
      S[q] = s;
    }
  }
  st.put(b, off, S[0]);
}

// ---- synthesis pass: Eq. (1)-ordered coefficients -> spatial block ---------
template <typename T, int V, int LI, int LO, LiftKind K>
__global__ __launch_bounds__(kThreads) void lift_synthesis(const T* __restrict__ in,
                                                           T* __restrict__ out, int64_t P,
                                                           int64_t p, int64_t nvec,
                                                           int64_t nblk_pos) {
  using Op = Level<K>;
  constexpr int L = LI + LO;
  constexpr int NI = 1 << LI;
  constexpr int NO = 1 << LO;
  const int64_t b = blockIdx.x / nblk_pos;
  const int64_t e = (blockIdx.x % nblk_pos) * kThreads + threadIdx.x;
  if (e >= nvec) return;
  const int64_t off = e * V;

  Pack<T, V> S[NO];
  S[0] = load_pack<T, V>(in + b * P + off);
#pragma unroll
  for (int jo = LO; jo >= 1; --jo) {
    const int j = LI + jo;
    const int cnt = NO >> jo;
    const int64_t dbase = (p >> j) + b * (int64_t(1) << (L - j));
#pragma unroll
    for (int q = cnt - 1; q >= 0; --q) {
      const Pack<T, V> d = load_pack<T, V>(in + (dbase + q) * P + off);
      Pack<T, V> x0, x1;
      apply_pair<T, V, Op>(S[q], d, x0, x1);
      S[2 * q] = x0;
      S[2 * q + 1] = x1;
    }
  }
#pragma unroll
  for (int sb = 0; sb < NO; ++sb) {
    Pack<T, V> v[NI];
    v[0] = S[sb];
#pragma unroll
    for (int j = LI; j >= 1; --j) {
      const int cnt = NI >> j;
      const int64_t dbase = (p >> j) + b * (int64_t(1) << (L - j)) + int64_t(sb) * cnt;
#pragma unroll
      for (int q = cnt - 1; q >= 0; --q) {
        const Pack<T, V> d = load_pack<T, V>(in + (dbase + q) * P + off);
        Pack<T, V> x0, x1;
        apply_pair<T, V, Op>(v[q], d, x0, x1);
        v[2 * q] = x0;
        v[2 * q + 1] = x1;
      }
    }
    const int64_t base = b * (NI * NO) + sb * NI;
#pragma unroll
    for (int t = 0; t < NI; ++t) store_pack<T, V>(out + (base + t) * P + off, v[t]);
  }
}

// ---- tiering and vector width ---------------------------------------------
constexpr int inner_levels(int L) { return L <= 4 ? L : (L <= 8 ? 4 : 5); }

// Widest vector (16 B) that keeps the block's live values within ~96 VGPRs.
template <typename T>
constexpr int pref_vec(int L) {
  const int li = inner_levels(L);
  const int regs = (1 << li) + (1 << (L - li));
  int v = 16 / int(sizeof(T));
  while (v > 1 && regs * v * int(sizeof(T)) / 4 > 96) v /= 2;
  return v;
}

struct Geometry {
  int64_t nvec, nblk_pos, grid;
};

inline Geometry geometry(int64_t P, int64_t p, int L, int V) {
  Geometry g;
  g.nvec = P / V;
  g.nblk_pos = (g.nvec + kThreads - 1) / kThreads;
  g.grid = g.nblk_pos * (p >> L);
  return g;
}

inline bool aligned(const void* ptr, size_t a) {
  return (reinterpret_cast<uintptr_t>(ptr) % a) == 0;
}

template <typename T, int V, int L, LiftKind K, class Store>
hipError_t run_analysis(const T* in, Store st, int64_t P, int64_t p, hipStream_t s) {
  constexpr int LI = inner_levels(L);
  const Geometry g = geometry(P, p, L, V);
  if (g.grid <= 0) return hipSuccess;
  if (g.grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((lift_analysis<T, V, LI, L - LI, K, Store>), dim3(unsigned(g.grid)),
                     dim3(kThreads), 0, s, in, st, P, p, g.nvec, g.nblk_pos);
  return hipGetLastError();
}

template <typename T, int V, int L, LiftKind K>
hipError_t run_synthesis(const T* in, T* out, int64_t P, int64_t p, hipStream_t s) {
  constexpr int LI = inner_levels(L);
  const Geometry g = geometry(P, p, L, V);
  if (g.grid <= 0) return hipSuccess;
  if (g.grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((lift_synthesis<T, V, LI, L - LI, K>), dim3(unsigned(g.grid)),
                     dim3(kThreads), 0, s, in, out, P, p, g.nvec, g.nblk_pos);
  return hipGetLastError();
}

// Plain-output passes for one compile-time level count.
template <typename T, int L>
hipError_t lift_plain_L(LiftKind kind, const T* in, T* out, int64_t P, int64_t p, hipStream_t s) {
  constexpr int VP = pref_vec<T>(L);
  const bool wide = (P % VP == 0) && aligned(in, sizeof(T) * VP) && aligned(out, sizeof(T) * VP);
  switch (kind) {
    case LiftKind::kForward:
      return wide ? run_analysis<T, VP, L, LiftKind::kForward>(in, PlainStore<T, VP>{out, P}, P, p, s)
                  : run_analysis<T, 1, L, LiftKind::kForward>(in, PlainStore<T, 1>{out, P}, P, p, s);
    case LiftKind::kInverseAdj:
      return wide ? run_analysis<T, VP, L, LiftKind::kInverseAdj>(in, PlainStore<T, VP>{out, P}, P, p, s)
                  : run_analysis<T, 1, L, LiftKind::kInverseAdj>(in, PlainStore<T, 1>{out, P}, P, p, s);
    case LiftKind::kInverse:
      return wide ? run_synthesis<T, VP, L, LiftKind::kInverse>(in, out, P, p, s)
                  : run_synthesis<T, 1, L, LiftKind::kInverse>(in, out, P, p, s);
    case LiftKind::kForwardAdj:
      return wide ? run_synthesis<T, VP, L, LiftKind::kForwardAdj>(in, out, P, p, s)
                  : run_synthesis<T, 1, L, LiftKind::kForwardAdj>(in, out, P, p, s);
  }
  return hipErrorInvalidValue;
}

template <int L>
hipError_t lift_split_L(LiftKind kind, const float* in, uint16_t* hi, uint16_t* lo, int64_t P,
                        int64_t p, hipStream_t s) {
  constexpr int VP = pref_vec<float>(L);
  const bool wide = (P % VP == 0) && aligned(in, 4 * VP) && aligned(hi, 2 * VP) &&
                    (lo == nullptr || aligned(lo, 2 * VP));
  switch (kind) {
    case LiftKind::kForward:
      return wide ? run_analysis<float, VP, L, LiftKind::kForward>(in, SplitStore<VP>{hi, lo, P}, P, p, s)
                  : run_analysis<float, 1, L, LiftKind::kForward>(in, SplitStore<1>{hi, lo, P}, P, p, s);
    case LiftKind::kInverseAdj:
      return wide ? run_analysis<float, VP, L, LiftKind::kInverseAdj>(in, SplitStore<VP>{hi, lo, P}, P, p, s)
                  : run_analysis<float, 1, L, LiftKind::kInverseAdj>(in, SplitStore<1>{hi, lo, P}, P, p, s);
    default:
      return hipErrorInvalidValue;  // synthesis passes produce spatial data, never split
  }
}

template <typename T>
hipError_t lift_plain(LiftKind kind, const T* in, T* out, int64_t P, int64_t p, int L,
                      hipStream_t s) {
  switch (L) {
    case 0: return lift_plain_L<T, 0>(kind, in, out, P, p, s);
    case 1: return lift_plain_L<T, 1>(kind, in, out, P, p, s);
    case 2: return lift_plain_L<T, 2>(kind, in, out, P, p, s);
    case 3: return lift_plain_L<T, 3>(kind, in, out, P, p, s);
    case 4: return lift_plain_L<T, 4>(kind, in, out, P, p, s);
    case 5: return lift_plain_L<T, 5>(kind, in, out, P, p, s);
    case 6: return lift_plain_L<T, 6>(kind, in, out, P, p, s);
    case 7: return lift_plain_L<T, 7>(kind, in, out, P, p, s);
    case 8: return lift_plain_L<T, 8>(kind, in, out, P, p, s);
    case 9: return lift_plain_L<T, 9>(kind, in, out, P, p, s);
    case 10: return lift_plain_L<T, 10>(kind, in, out, P, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_lift_f64(LiftKind kind, const double* in, double* out, int64_t P, int64_t p,
                           int L, hipStream_t s) {
  return lift_plain<double>(kind, in, out, P, p, L, s);
}

hipError_t launch_lift_f32(LiftKind kind, const float* in, float* out, int64_t P, int64_t p,
                           int L, hipStream_t s) {
  return lift_plain<float>(kind, in, out, P, p, L, s);
}

hipError_t launch_lift_f32_split(LiftKind kind, const float* in, uint16_t* hi, uint16_t* lo,
                                 int64_t P, int64_t p, int L, hipStream_t s) {
  switch (L) {
    case 0: return lift_split_L<0>(kind, in, hi, lo, P, p, s);
    case 1: return lift_split_L<1>(kind, in, hi, lo, P, p, s);
    case 2: return lift_split_L<2>(kind, in, hi, lo, P, p, s);
    case 3: return lift_split_L<3>(kind, in, hi, lo, P, p, s);
    case 4: return lift_split_L<4>(kind, in, hi, lo, P, p, s);
    case 5: return lift_split_L<5>(kind, in, hi, lo, P, p, s);
    case 6: return lift_split_L<6>(kind, in, hi, lo, P, p, s);
    case 7: return lift_split_L<7>(kind, in, hi, lo, P, p, s);
    case 8: return lift_split_L<8>(kind, in, hi, lo, P, p, s);
    case 9: return lift_split_L<9>(kind, in, hi, lo, P, p, s);
    case 10: return lift_split_L<10>(kind, in, hi, lo, P, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace wp
