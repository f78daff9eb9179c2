// w-svd (Alg. 2, Thm 2.5) for gfx950: per-coefficient-slice truncated SVD by
// one-sided (Hestenes) Jacobi, rank-k rebuild on the face-product GEMM, and
// the inverse lifting.
//
// Jacobi: a coefficient slice is viewed as a matrix W with mr = max(n1, n2)
// rows and nc = min(n1, n2) columns (the slice itself when n1 >= n2, its
// transpose otherwise).  A sweep visits every column pair once, as a
// round-robin tournament: nc_pad - 1 rounds of nc_pad / 2 disjoint pairs.  For
// each pair gamma = w_i.w_j is summed in the data type (FP32 lane partials and
// FP32 cross-lane sums for FP32 data, FP64 throughout for FP64 data; FP64 sums
// of FP32 data measured 1.6x slower for the same sweeps and errors); the
// squared norms alpha = |w_i|^2, beta = |w_j|^2 are summed the same way when a
// sweep (register kernel) or a launch (block kernel) starts and then carried
// with the columns through the rotations (alpha - t gamma, beta + t gamma).
// When |gamma| > tol * sqrt(alpha * beta) (tol = sqrt(mr) * unit roundoff of
// the data type) the rotation parameters are computed in FP64 and the
// rotation is applied to columns i, j of W in the data type.  A slice has
// converged after a sweep without rotation.
//
// Register-resident kernel (the columns of a slice fit the registers of one
// workgroup): 32 units of 16 lanes each hold J tournament slots (a top and a
// bottom column per slot), rows spread over the unit's lanes.  alpha, beta,
// gamma are row sums inside a unit (DPP), the J angles of a unit are
// evaluated side by side in FP64 and broadcast, and the circle advance of
// the round-robin tournament is a renaming of register slots plus two
// columns per unit through LDS.  Only W is kept; the second factor is
// recovered from A V = U Sigma afterwards and orthonormalised.  A block
// kernel spreads a slice over many workgroups and covers the larger shapes
// and the calls with few slices; it keeps only W as well.
//
// sp-w-svd (Sec. IV-B) runs the same kernels on the s_L and d_L slices only
// and leaves the finer details zero in the rebuild.
//
// Afterwards sigma_i = |w_i| (FP64), the columns are ranked by decreasing
// sigma (ties by index), the k leading ones are normalised into U, signs are
// fixed so that each U column's largest-magnitude entry is positive, and
// U * sigma is written for the rebuild.

#include <type_traits>

#include "wp_internal.h"

namespace wp {
namespace {

constexpr int kJacobiWaves = 8;
constexpr int kJacobiThreads = 64 * kJacobiWaves;
// Largest slice side handled (rows and columns of W).
constexpr int kMaxSide = 2048;

template <typename T>
struct Unit;
template <>
struct Unit<float> {
  static constexpr double value = 5.9604644775390625e-08;  // 2^-24
};
template <>
struct Unit<double> {
  static constexpr double value = 1.1102230246251565e-16;  // 2^-53
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Round-robin tournament: in round r of n players (n even), pair q is
// (n-1, r) for q = 0 and ((r+q) mod (n-1), (r-q) mod (n-1)) otherwise.
__device__ __forceinline__ void rr_pair(int n, int r, int q, int& i, int& j) {
  if (q == 0) {
    i = n - 1;
    j = r;
  } else {
    i = (r + q) % (n - 1);
    j = (r - q + (n - 1)) % (n - 1);
  }
}

struct SvdDims {
  int n1, n2, mr, nc, ncp, k;
  int trans;  // W = slice^T (n1 < n2)
};

// FP64 reciprocal and reciprocal square root from the hardware estimates
// (v_rcp_f64 / v_rsq_f64, ~5e-8 relative) refined by NS Newton steps, each of
// which doubles the number of correct bits: measured on gfx950 over 2^20
// arguments, one step leaves 4e-15 (rsq) and 2e-15 (rcp), two 2.4e-16 and
// 1.1e-16, about one unit in the last place; no scaling and fix-up sequences
// as in the correctly rounded library routines.  Arguments are finite and
// positive.
template <int NS>
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
  }
  return r;
}
template <int NS>
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
#pragma unroll
  for (int i = 0; i < NS; ++i) y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Newton steps of the rotation parameters for data of type T: FP64 data get
// parameters accurate to the last place; for FP32 data, whose rotations are
// applied in FP32, one step leaves them accurate to ~4e-15.
template <typename T>
constexpr int kRotNewton = sizeof(T) == 8 ? 2 : 1;

// Rotation that zeroes w_i.w_j, evaluated in FP64.  With d = beta - alpha the
// tangent t = sign(d) * 2 gamma / (|d| + sqrt(d^2 + 4 gamma^2)) is the smaller
// root of t^2 + 2 zeta t - 1 = 0, zeta = d / (2 gamma) (Rutishauser's choice);
// c = 1 / sqrt(1 + t^2), s = c t.  The tangent is returned too, for updating
// the two column norms: with gamma zeroed, |w_i'|^2 = alpha - t gamma and
// |w_j'|^2 = beta + t gamma.
// Returns 0: below the threshold (c = 1, s = t = 0), 1: rotate, 2: non-finite
// input.
template <int NS>
__device__ __forceinline__ int rotation_t(double al, double be, double ga, double tol, double& c,
                                          double& s, double& t) {
  c = 1.0;
  s = 0.0;
  t = 0.0;
  if (!(isfinite(al) && isfinite(be) && isfinite(ga))) return 2;
  if (!(ga * ga > tol * tol * (al * be))) return 0;
  // Here gamma != 0, so q > 0 and every argument below is positive.
  const double d = be - al;
  const double g2 = 2.0 * ga;
  const double q = fma(d, d, g2 * g2);
  const double h = q * rsqrt64<NS>(q);
  t = copysign(1.0, d) * g2 * rcp64<NS>(fabs(d) + h);
  c = rsqrt64<NS>(fma(t, t, 1.0));
  s = c * t;
  return 1;
}

// Ranks the nc columns by a strict total order: larger sigma first, NaN after
// every number, ties (and NaNs) by column index; the ranks are therefore a
// permutation.  s_order[rank] = column, and s_rank[column] = rank when s_rank
// is given.  Called by every thread of the workgroup.
__device__ void rank_columns(int nc, const double* s_sigma, int* s_order, int* s_rank) {
  for (int c = threadIdx.x; c < nc; c += kJacobiThreads) {
    const double sc = s_sigma[c];
    const bool nan_c = sc != sc;
    int rank = 0;
    for (int o = 0; o < nc; ++o) {
      const double so = s_sigma[o];
      const bool nan_o = so != so;
      const bool before = nan_o ? (nan_c && o < c)
                                : (nan_c || so > sc || (so == sc && o < c));
      rank += before;
    }
    s_order[rank] = c;
    if (s_rank != nullptr) s_rank[c] = rank;
  }
}

// emit_factors for the register-resident kernel, from the columns still in
// registers (unit of 16 lanes, rows lane16 + 16 t; column ids ct[j], cb[j] of
// the J top and bottom slots, nc for none), after rank_columns.  The k
// leading columns go to LDS as they are (`cap` values at s_col, as many
// columns at a time as fit; their signs at s_sgn), then are normalised (and
// sign-fixed when they form U) in FP64 while written out row by row.
template <typename T, int J, int RPL>
__device__ __forceinline__ void emit_from_registers(const T (&tc)[J][RPL], const T (&bc)[J][RPL],
                                    const int (&ct)[J], const int (&cb)[J], const SvdDims& d,
                                    int slice, int lane16, const double* s_sigma,
                                    const int* s_order, const int* s_rank, int* s_sgn, T* s_col,
                                    int cap, T* __restrict__ uhat, T* __restrict__ shat,
                                    T* __restrict__ vhat, T* __restrict__ us) {
  const int mr = d.mr, nc = d.nc, k = d.k;
  T* U = uhat + int64_t(slice) * d.n1 * k;
  T* Vo = vhat + int64_t(slice) * d.n2 * k;
  T* Us = us + int64_t(slice) * d.n1 * k;
  // Columns staged at a time: the exchange buffers hold 4 kUnits slots of
  // 16 RPL + 16 >= mr + 16 values, so at least 128 columns fit next to the
  // rank and sign arrays.
  const int per = cap / mr;
  for (int i0 = 0; i0 < k; i0 += per) {
    const int i1 = i0 + per < k ? i0 + per : k;
    auto stage = [&](const T (&x)[RPL], int c) {
      if (c >= nc) return;
      const int i = s_rank[c];
      if (i < i0 || i >= i1) return;
      // Largest |entry|, lowest row on ties: its sign is the column's (U is
      // made positive there; w / sigma orders its entries as w does).
      T best = T(-1);
      int brow = 0x7fffffff, neg = 0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = lane16 + 16 * t;
        if (row < mr && fabs(x[t]) > best) {
          best = fabs(x[t]);
          brow = row;
          neg = x[t] < T(0);
        }
      }
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) {
        const T ob = __shfl_xor(best, o, 16);
        const int orow = __shfl_xor(brow, o, 16);
        const int on = __shfl_xor(neg, o, 16);
        if (ob > best || (ob == best && orow < brow)) {
          best = ob;
          brow = orow;
          neg = on;
        }
      }
      T* col = s_col + (i - i0) * mr;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = lane16 + 16 * t;
        if (row < mr) col[row] = x[t];
      }
      if (lane16 == 0) {
        s_sgn[i - i0] = neg;
        shat[int64_t(slice) * k + i] = T(s_sigma[c]);
      }
    };
#pragma unroll
    for (int j = 0; j < J; ++j) {
      stage(tc[j], ct[j]);
      stage(bc[j], cb[j]);
    }
    __syncthreads();
    const int w = i1 - i0;
    for (int e = threadIdx.x; e < mr * w; e += kJacobiThreads) {
      const int row = e / w, ii = e - row * w;
      const double sg = s_sigma[s_order[i0 + ii]];
      const double inv = sg > 0 ? 1.0 / sg : 0.0;
      const double v = double(s_col[ii * mr + row]) * inv;
      if (d.trans) {
        // W holds the transposed slice: w_c / sigma is a right singular vector.
        Vo[int64_t(row) * k + i0 + ii] = T(v);
      } else {
        const double x = s_sgn[ii] && sg > 0 ? -v : v;
        U[int64_t(row) * k + i0 + ii] = T(x);
        Us[int64_t(row) * k + i0 + ii] = T(T(x) * T(sg));
      }
    }
    __syncthreads();
  }
}

// Singular values, ranking and the k leading columns of the factor formed by
// W (column c at W + c * mr), called by every thread of the workgroup: U (and
// U * sigma) when n1 >= n2, vhat otherwise.  The other factor is recovered
// afterwards from the coefficients (recover_kernel), which in the second case
// also fixes the signs.
template <typename T>
__device__ void emit_factors(const T* __restrict__ W, const SvdDims& d, int slice,
                             T* __restrict__ uhat, T* __restrict__ shat, T* __restrict__ vhat,
                             T* __restrict__ us, double* s_sigma, int* s_order) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int mr = d.mr, nc = d.nc;
  for (int c = wave; c < nc; c += kJacobiWaves) {
    double acc = 0;
    for (int row = lane; row < mr; row += 64) {
      const double x = double(W[int64_t(c) * mr + row]);
      acc = fma(x, x, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) s_sigma[c] = sqrt(acc);
  }
  __syncthreads();
  rank_columns(nc, s_sigma, s_order, nullptr);
  __syncthreads();

  const int k = d.k;
  T* U = uhat + int64_t(slice) * d.n1 * k;
  T* Vo = vhat + int64_t(slice) * d.n2 * k;
  T* Us = us + int64_t(slice) * d.n1 * k;
  for (int i = wave; i < k; i += kJacobiWaves) {
    const int c = s_order[i];
    const double sg = s_sigma[c];
    const double inv = sg > 0 ? 1.0 / sg : 0.0;
    const T* w = W + int64_t(c) * mr;
    if (lane == 0) shat[int64_t(slice) * k + i] = T(sg);
    if (d.trans) {
      // W holds the transposed slice: w_c / sigma is a right singular vector.
      for (int row = lane; row < mr; row += 64) Vo[int64_t(row) * k + i] = T(double(w[row]) * inv);
      continue;
    }
    // Largest |U| entry, lowest row on ties, made positive.
    double best = -1.0;
    int brow = 0x7fffffff;
    double bval = 0;
    for (int row = lane; row < mr; row += 64) {
      const double x = double(w[row]) * inv;
      const double ax = fabs(x);
      if (ax > best) {
        best = ax;
        brow = row;
        bval = x;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int orow = __shfl_xor(brow, o, 64);
      const double ov = __shfl_xor(bval, o, 64);
      if (ob > best || (ob == best && orow < brow)) {
        best = ob;
        brow = orow;
        bval = ov;
      }
    }
    const double sgn = bval < 0 ? -1.0 : 1.0;
    for (int row = lane; row < mr; row += 64) {
      const double x = sgn * double(w[row]) * inv;
      U[int64_t(row) * k + i] = T(x);
      Us[int64_t(row) * k + i] = T(T(x) * T(sg));
    }
  }
}

// Cross-lane moves inside rows of 16 lanes.  CTRL is a DPP control word; all
// controls used here read a valid lane, so the moves need no old value.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T x) {
  if constexpr (sizeof(T) == 8)
    return dpp_f64<CTRL>(x);
  else
    return dpp_f32<CTRL>(x);
}

// Sum over the 16 lanes of a row: rotate by 8 and by 4 inside the row, then
// swap pairs of 2 and of 1 inside quads.  Each step adds two values in both
// partner lanes (a + b and b + a), so all 16 lanes end with the same bits.
// In FP32 the move is fused into the add (v_add_f32 with DPP).
template <typename T>
__device__ __forceinline__ T row_sum16(T x) {
  x += dpp_move<0x128>(x);  // row_ror:8
  x += dpp_move<0x124>(x);  // row_ror:4
  x += dpp_move<0x4e>(x);   // quad_perm [2,3,0,1]
  x += dpp_move<0xb1>(x);   // quad_perm [1,0,3,2]
  return x;
}

// Value of lane L of the row, in every lane of the row (row_newbcast).
template <int L, typename T>
__device__ __forceinline__ T row_bcast(T x) {
  return dpp_move<0x150 + L>(x);
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ---- Block one-sided Jacobi (slices beyond the register-resident kernel) ----
// W (mr x nc, column c at W + c * mr) is padded with zero columns to
// nbp * B columns, grouped in nbp blocks of B.  A sweep is a round-robin
// tournament over the blocks: nbp - 1 rounds of nbp / 2 block pairs, one
// launch per round and one workgroup per (block pair, slice), so a slice is
// spread over many compute units.  The workgroup holds its two blocks in
// registers: B groups of GL = 512 / B lanes, group g keeps column g of the
// first block and, in sub-round t, column (g + t) mod B of the second, which
// advances one group per sub-round through LDS; all B * B cross pairs are
// rotated.  In the first round of a sweep each block also rotates its own
// B (B - 1) / 2 pairs (round-robin over the block, columns in LDS), so every
// column pair of the slice is visited exactly once per sweep, with the same
// rotation and threshold as the one-workgroup kernel.  Per-slice control words
// count the rotations of a sweep; a slice stops (its later launches return at
// once) after a sweep without rotation, on a non-finite value, or after the
// sweep limit.  Only W is kept; the second factor is recovered afterwards.

constexpr int kBjThreads = 512;

struct BjCtl {
  int state;   // 0 running, 1 converged, 2 non-finite value, 3 out of sweeps
  int sweeps;  // sweeps completed
  int rot;     // rotations in the current sweep
  int bad;     // non-finite value seen in the current sweep
  int live;    // the slice has a nonzero entry (a zero slice needs no rotation)
  int pad[3];
};

// Block width and rows per lane of the block kernel for mr rows.
struct BjShape {
  int B, rpl, nbp;
};
inline BjShape bj_shape(int mr, int nc) {
  BjShape s{};
  s.B = mr <= 1024 ? 16 : 8;
  const int gl = kBjThreads / s.B;
  s.rpl = ((mr + gl - 1) / gl + 3) / 4 * 4;
  const int nb = (nc + s.B - 1) / s.B;
  s.nbp = nb + (nb & 1);
  return s;
}

// Sum over an aligned group of GL = 32 or 64 lanes, the same bits in every
// lane: 16-lane row sums (DPP), then the partner row (permlane16_swap) and
// for 64 lanes the partner half (permlane32_swap).  With a = b = x a swap
// leaves the even (lower) part's value in a and the odd (upper) part's in b
// on both sides, so every lane adds the two in the same order.
template <bool HALF>
__device__ __forceinline__ void swap_parts(unsigned& a, unsigned& b) {
  if constexpr (HALF) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  }
}
template <bool HALF>
__device__ __forceinline__ double pair_sum(double x) {
  unsigned lo0 = unsigned(__double2loint(x)), hi0 = unsigned(__double2hiint(x));
  unsigned lo1 = lo0, hi1 = hi0;
  swap_parts<HALF>(lo0, lo1);
  swap_parts<HALF>(hi0, hi1);
  return __hiloint2double(int(hi0), int(lo0)) + __hiloint2double(int(hi1), int(lo1));
}
template <bool HALF>
__device__ __forceinline__ float pair_sum(float x) {
  unsigned a = __builtin_bit_cast(unsigned, x), b = a;
  swap_parts<HALF>(a, b);
  return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}
template <int GL, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(GL == 32 || GL == 64, "group of 32 or 64 lanes");
  v = row_sum16<T>(v);
  v = pair_sum<false>(v);
  if constexpr (GL == 64) v = pair_sum<true>(v);
  return v;
}

// Copies the slices into column-major W through 32 x 32 LDS tiles (coalesced
// on both sides for either orientation), zeroes the padding columns and marks
// the slices that have a nonzero entry.
template <typename T>
__global__ __launch_bounds__(256) void bj_init_kernel(const T* __restrict__ ah,
                                                      T* __restrict__ wbuf, SvdDims d, int ncb,
                                                      BjCtl* __restrict__ ctl) {
  __shared__ T tile[32][33];
  const int slice = blockIdx.z;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const T* a = ah + int64_t(slice) * d.n1 * d.n2;
  T* W = wbuf + int64_t(slice) * ncb * d.mr;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // W[r][c] = slice (r, c) when not transposed (read along c), (c, r) otherwise
  // (read along r); tile[r - r0][c - c0].
  for (int y = ty; y < 32; y += 8) {
    if (d.trans) {
      const int r = r0 + tx, c = c0 + y;
      tile[tx][y] = (r < d.mr && c < d.nc) ? a[int64_t(c) * d.n2 + r] : T(0);
    } else {
      const int r = r0 + y, c = c0 + tx;
      tile[y][tx] = (r < d.mr && c < d.nc) ? a[int64_t(r) * d.n2 + c] : T(0);
    }
  }
  __syncthreads();
  bool nz = false;
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + tx, c = c0 + y;
    const T v = tile[tx][y];
    nz |= v != T(0);  // NaN counts as nonzero
    if (r < d.mr && c < ncb) W[int64_t(c) * d.mr + r] = v;
  }
  if (__syncthreads_or(nz) && threadIdx.x == 0) atomicOr(&ctl[slice].live, 1);
}

template <typename T, int B, int RPL>
__global__ __launch_bounds__(kBjThreads) void bj_round_kernel(T* __restrict__ wbuf, int mr,
                                                              int nbp, int round,
                                                              BjCtl* __restrict__ ctl,
                                                              double tol) {
  constexpr int GL = kBjThreads / B;  // lanes per group
  constexpr int CAP = GL * RPL;       // rows per column slot
  // Room for both blocks in LDS where that takes at most 40 KiB: the first
  // round then rotates the inner pairs of the two blocks side by side, and
  // the cross sub-rounds alternate between two exchange buffers.
  constexpr bool kTwo = 2 * B * CAP * int(sizeof(T)) <= 40 * 1024;
  __shared__ T s_x[(kTwo ? 2 : 1) * B * CAP];
  __shared__ double s_n[(kTwo ? 2 : 1) * B];  // squared norms of the columns in the LDS slots
  const int slice = blockIdx.y;
  if (ctl[slice].state != 0 || !ctl[slice].live) return;
  int bi, bj;
  rr_pair(nbp, round, blockIdx.x, bi, bj);
  T* W = wbuf + int64_t(slice) * nbp * B * mr;
  const int g = threadIdx.x / GL;
  const int l = threadIdx.x % GL;
  int nrot = 0;
  bool bad = false;

  auto norm2 = [&](const T (&x)[RPL]) -> double {
    T a = 0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) a = fma(x[t], x[t], a);
    return double(group_sum<GL>(a));
  };
  // Rotation for the pair (x, y) (this lane's rows): gamma from the group's
  // sum, the squared norms al, be carried with the columns and updated to
  // those of the rotated pair (al - t gamma, be + t gamma).
  auto angle = [&](const T (&x)[RPL], const T (&y)[RPL], double& al, double& be, double& c,
                   double& s) {
    T ga = 0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) ga = fma(x[t], y[t], ga);
    const double g64 = double(group_sum<GL>(ga));
    double tt;
    const int f = rotation_t<kRotNewton<T>>(al, be, g64, tol, c, s, tt);
    al = fma(-tt, g64, al);
    be = fma(tt, g64, be);
    nrot += f == 1;
    bad |= f == 2;
  };

  T top[RPL], bot[RPL];
  double ntop, nbot;
  if (round == 0) {
    // Pairs inside each block: columns in LDS slots, B / 2 groups per block
    // rotate one pair each per sub-round, streaming the two columns from LDS
    // (once for gamma, once more to rotate) so that only the other block's
    // columns stay in registers.  With two buffers both blocks run side by
    // side (groups B / 2 .. B - 1 take block I), otherwise J first, then I.
    constexpr int kPar = kTwo ? 2 : 1;
#pragma unroll
    for (int pass = 0; pass < 2 / kPar; ++pass) {
#pragma unroll
      for (int h = 0; h < kPar; ++h) {
        const int blk = pass * kPar + h;  // 0: block J, 1: block I
        const T* src = W + int64_t((blk == 0 ? bj : bi) * B + g) * mr;
        T* dst = s_x + h * B * CAP + g * CAP + l;
        T a = 0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int row = l + GL * t;
          const T v = row < mr ? src[row] : T(0);
          dst[GL * t] = v;
          a = fma(v, v, a);
        }
        a = group_sum<GL>(a);
        if (l == 0) s_n[h * B + g] = double(a);
      }
      __syncthreads();
      const int h = g / (B / 2);
      for (int r = 0; r < B - 1; ++r) {
        if (h < kPar) {
          int i, j;
          rr_pair(B, r, g % (B / 2), i, j);
          T* xi = s_x + h * B * CAP + i * CAP + l;
          T* xj = s_x + h * B * CAP + j * CAP + l;
          double* ni = s_n + h * B + i;
          double* nj = s_n + h * B + j;
          T ga = 0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) ga = fma(xi[GL * t], xj[GL * t], ga);
          const double g64 = double(group_sum<GL>(ga));
          double al = *ni, be = *nj, c, sn, tt;
          const int f = rotation_t<kRotNewton<T>>(al, be, g64, tol, c, sn, tt);
          nrot += f == 1;
          bad |= f == 2;
          if (f == 1) {
            const T ct = T(c), st = T(sn);
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              const T x = xi[GL * t], y = xj[GL * t];
              xi[GL * t] = ct * x - st * y;
              xj[GL * t] = st * x + ct * y;
            }
            if (l == 0) {
              *ni = fma(-tt, g64, al);
              *nj = fma(tt, g64, be);
            }
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int hh = 0; hh < kPar; ++hh) {
        const int blk = pass * kPar + hh;
        const T* src = s_x + hh * B * CAP + g * CAP + l;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          if (blk == 0)
            bot[t] = src[GL * t];
          else
            top[t] = src[GL * t];
        }
        if (blk == 0)
          nbot = s_n[hh * B + g];
        else
          ntop = s_n[hh * B + g];
      }
      __syncthreads();
    }
  } else {
    const T* ti = W + int64_t(bi * B + g) * mr;
    const T* tj = W + int64_t(bj * B + g) * mr;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = l + GL * t;
      top[t] = row < mr ? ti[row] : T(0);
      bot[t] = row < mr ? tj[row] : T(0);
    }
    ntop = norm2(top);
    nbot = norm2(bot);
  }

  // Cross pairs: group g holds column g of block bi and, in sub-round t,
  // column (g + t) mod B of block bj, which carries its squared norm along.
  for (int sub = 0; sub < B; ++sub) {
    double c, s;
    angle(top, bot, ntop, nbot, c, s);
    const T ct = T(c), st = T(s);
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const T x = top[t], y = bot[t];
      top[t] = ct * x - st * y;
      bot[t] = st * x + ct * y;
    }
    if (sub + 1 < B) {
      // Group g passes its column to group g - 1 and takes group g + 1's, with
      // one barrier between the writes and the reads.  With room for two
      // buffers, sub-round t uses buffer t mod 2 (a group writes it again only
      // after the next barrier, which every group reaches after its reads);
      // with one, group g writes slot (g + t) mod B and reads slot
      // (g + 1 + t) mod B, so the slot it writes next is the one it has just
      // read itself.  (Both measured: the first is ~2 % faster where it fits.)
      int ws, rs;
      T* xb = s_x;
      double* nb = s_n;
      if constexpr (kTwo) {
        xb += (sub & 1) * B * CAP;
        nb += (sub & 1) * B;
        ws = g;
        rs = (g + 1) % B;
      } else {
        ws = (g + sub) % B;
        rs = (g + 1 + sub) % B;
      }
#pragma unroll
      for (int t = 0; t < RPL; ++t) xb[ws * CAP + GL * t + l] = bot[t];
      if (l == 0) nb[ws] = nbot;
      __syncthreads();
#pragma unroll
      for (int t = 0; t < RPL; ++t) bot[t] = xb[rs * CAP + GL * t + l];
      nbot = nb[rs];
    }
  }
  T* di = W + int64_t(bi * B + g) * mr;
  T* dj = W + int64_t(bj * B + (g + B - 1) % B) * mr;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int row = l + GL * t;
    if (row < mr) {
      di[row] = top[t];
      dj[row] = bot[t];
    }
  }
  if (l == 0 && nrot > 0) atomicAdd(&ctl[slice].rot, nrot);
  if (l == 0 && bad) atomicOr(&ctl[slice].bad, 1);
}

// End of a sweep: count it and decide whether each slice goes on.
__global__ __launch_bounds__(256) void bj_sweep_end_kernel(BjCtl* __restrict__ ctl, int nsl,
                                                           int max_sweeps) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= nsl) return;
  BjCtl c = ctl[s];
  if (c.state != 0) return;
  c.sweeps += 1;
  if (c.bad)
    c.state = 2;
  else if (c.rot == 0)
    c.state = 1;
  else if (c.sweeps >= max_sweeps)
    c.state = 3;
  c.rot = 0;
  ctl[s] = c;
}

// Singular values, ranking and the factor taken from W, per slice.
template <typename T>
__global__ __launch_bounds__(kJacobiThreads) void bj_emit_kernel(
    const T* __restrict__ wbuf, SvdDims d, int ncb, const BjCtl* __restrict__ ctl,
    T* __restrict__ uhat, T* __restrict__ shat, T* __restrict__ vhat, T* __restrict__ us,
    int32_t* __restrict__ info) {
  __shared__ double s_sigma[kMaxSide];
  __shared__ int s_order[kMaxSide];
  const int slice = blockIdx.x;
  emit_factors<T>(wbuf + int64_t(slice) * ncb * d.mr, d, slice, uhat, shat, vhat, us, s_sigma,
                  s_order);
  if (threadIdx.x == 0) {
    const BjCtl c = ctl[slice];
    info[slice] = c.state == 1 ? c.sweeps : -(c.sweeps > 0 ? c.sweeps : 1);
  }
}

constexpr int kUnits = 4 * kJacobiWaves;  // 16-lane rows per workgroup
// Blocks of J rounds between two foldings of the column scales (register kernel).
constexpr int kRescaleBlocks = 16;

// Register-resident Jacobi on W only.  A unit is one 16-lane DPP row; column
// entries are spread over its lanes, RPL rows per lane (row = lane16 + 16 t,
// mr <= 16 * RPL).  Unit u owns the J consecutive tournament slots uJ..uJ+J-1
// (a top and a bottom column each), so a wavefront works on 4 J pairs per
// round.  nunits * J slots in total; positions beyond nc hold zero columns,
// which never rotate.
//
// Per round and pair: gamma as a 16-lane row sum (FP32 data: FP32 lane
// partials and FP32 row sums, at most RPL + 4 rounding steps; FP64 data: FP64
// throughout); the two column norms alpha, beta are not summed again but
// carried with the columns: each column's squared norm is kept in FP64 (in
// LDS, by column), summed exactly at the start of every sweep and updated
// after each rotation by alpha - t gamma, beta + t gamma (exact for the
// rotation that zeroes gamma).  That saves two of the three dot products of
// a pair.  Kept in FP32 instead, the rounding of every update drifts the
// norms enough within a sweep to cost the slowest slice of the
// hyperspectral-like test tensor one more sweep.  The J angles of a unit are
// evaluated together in FP64, pair j in lanes j (16 / J) .., and the shear
// factors are broadcast to the row.
//
// Circle method: position 0 (unit 0, top slot 0) is fixed and the other
// positions advance one step per round (top q -> top q+1, top H-1 -> bottom
// H-1, bottom q -> bottom q-1, bottom 0 -> top 1).  Inside a unit this is a
// renaming of the J register slots, so the round loop is unrolled J times and
// at unrolled step rr logical top j lives in register slot (j - rr) mod J and
// logical bottom j in slot (j + rr) mod J.  Only the unit's last top and
// first bottom column leave it, through LDS, into the slots that they vacate.
// Unit 0 also passes its fixed column through LDS and takes its own first
// bottom column into top slot 1.
template <typename T, int J, int RPL>
__global__ __launch_bounds__(kJacobiThreads) void jacobi_reg_kernel(
    const T* __restrict__ ah, SvdDims d, int nunits, int max_sweeps, T* __restrict__ uhat,
    T* __restrict__ shat, T* __restrict__ vhat, T* __restrict__ us, int32_t* __restrict__ info) {
  static_assert(J == 1 || J == 2 || J == 4, "J is 1, 2 or 4");
  constexpr int M = J - 1;
  constexpr int SLOT = 16 * RPL + 16;  // padding puts the 4 units of a wave on other banks
  constexpr int PAR = 2 * kUnits * SLOT;
  const int slice = blockIdx.x;
  const int lane16 = threadIdx.x & 15;
  const int unit = threadIdx.x >> 4;
  const int mr = d.mr, nc = d.nc;
  const int H = nunits * J;
  const int CIRC = 2 * H - 1;
  const bool active = unit < nunits;
  const int last = nunits - 1;
  const int q0 = unit * J;
  const T* a = ah + int64_t(slice) * d.n1 * d.n2;

  // [round parity][outgoing top, outgoing bottom][unit][row]
  __shared__ T s_x[2][2][kUnits][SLOT];
  __shared__ T s_fx[2][SLOT];  // unit 0's fixed column
  __shared__ int s_rot[2];
  __shared__ int s_bad;
  __shared__ double s_sigma[1024];
  __shared__ int s_order[1024];
  // Squared norm of every column (carried in FP64), indexed by column (the columns move
  // between units, their norms stay in place); shares the storage of the
  // singular values, which are formed only after the sweeps.
  // With them, the scales d of the columns (w = d x) and their inverses e,
  // indexed the same way.
  constexpr int kPos = 2 * kUnits * 4;
  static_assert(kPos * 3 * sizeof(double) <= sizeof(s_sigma), "fits");
  double* const s_d = s_sigma;
  double* const s_e = s_sigma + kPos;
  double* const s_norm = s_sigma + 2 * kPos;

  // Column held by slot q after r rounds (0 <= r < CIRC): position p starts
  // with column p and the circle advances one position per round.
  // (0 <= q-1, 2H-2-q < CIRC, so one conditional wrap suffices.)
  auto wrap = [&](int x) { return (x < 0 ? x + CIRC : x) + 1; };
  auto top_id = [&](int q, int r) { return q == 0 ? 0 : wrap(q - 1 - r); };
  auto bot_id = [&](int q, int r) { return wrap(2 * H - 2 - q - r); };
  auto w_src = [&](int row, int c) -> T {
    return d.trans ? a[c * d.n2 + row] : a[row * d.n2 + c];
  };

  // Where the columns entering this unit come from (parity 0 addresses).
  // New top 0: unit 0 keeps its fixed column; with J == 1 unit 1 takes unit
  // 0's first bottom; otherwise the left neighbour's last top.  New bottom
  // J-1: the right neighbour's first bottom; the last unit takes its own
  // last top (its own first bottom when H == 1, where nothing moves).
  // Units past the last one hold zero columns and read back their own
  // outgoing (zero) columns, so they never rotate.
  const T* in_top;
  int in_top_par = PAR;
  const T* in_bot;
  if (!active) {
    in_top = &s_x[0][0][unit][0];
    in_bot = &s_x[0][1][unit][0];
  } else {
    if (unit == 0) {
      in_top = &s_fx[0][0];
      in_top_par = SLOT;
    } else {
      in_top = (J == 1 && unit == 1) ? &s_x[0][1][0][0] : &s_x[0][0][unit - 1][0];
    }
    in_bot = unit < last ? &s_x[0][1][unit + 1][0]
                         : (H == 1 ? &s_x[0][1][unit][0] : &s_x[0][0][unit][0]);
  }
  // Every unit runs the same instructions (no branch around the round body,
  // which keeps the renamed register slots in place); a wavefront without an
  // active unit works on zero columns.
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));

  T tc[J][RPL], bc[J][RPL];
  // Columns of a row-major slice (no transpose) are strided in memory, and
  // gathering them lane by lane fetches each line many times over; they go
  // through LDS instead, half the rows at a time: coalesced row reads into
  // the (not yet used) exchange buffer, then each lane picks its entries.
  constexpr int CH = 8 * RPL;  // rows per half
  const int ld = nc + 1;       // odd pitch: a unit's 16 rows hit 16 banks
  const bool staged = !d.trans && RPL >= 2 &&
                      CH * ld <= int(sizeof(s_x) / sizeof(T));
  if (staged) {
    T* stage = &s_x[0][0][0][0];
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int r0 = half * CH;
      for (int r = wave; r < CH; r += kJacobiWaves) {
        const bool in = r0 + r < mr;
        for (int c = lane; c < nc; c += 64) stage[r * ld + c] = in ? a[(r0 + r) * d.n2 + c] : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int it = top_id(q0 + j, 0), ib = bot_id(q0 + j, 0);
#pragma unroll
        for (int t = half * (RPL / 2); t < (half + 1) * (RPL / 2); ++t) {
          const int row = lane16 + 16 * t;
          const bool ok = active && row < mr;
          const int lr = row - r0;  // in [0, CH)
          const T vt = stage[lr * ld + (it < nc ? it : 0)];
          const T vb = stage[lr * ld + (ib < nc ? ib : 0)];
          tc[j][t] = (ok && it < nc) ? vt : T(0);
          bc[j][t] = (ok && ib < nc) ? vb : T(0);
        }
      }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int it = top_id(q0 + j, 0), ib = bot_id(q0 + j, 0);
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = lane16 + 16 * t;
        const bool ok = active && row < mr;
        tc[j][t] = (ok && it < nc) ? w_src(row, it) : T(0);
        bc[j][t] = (ok && ib < nc) ? w_src(row, ib) : T(0);
      }
    }
  }
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_rot[0] = 0;
    s_rot[1] = 0;
  }
  __syncthreads();

  const double tol = sqrt(double(mr)) * Unit<T>::value;
  int sw = 0, par = 0, my_rot = 0;
  bool my_bad = false, converged = false;

  // A sweep runs 2H = CIRC + 1 rounds, a whole number of J-round blocks, so
  // the register renaming is the identity at every sweep end (the extra
  // round repeats the pairs of the sweep's first round).
  // The 16 / J lanes j (16 / J) .. of a unit evaluate the angle of the unit's
  // pair j (top position q0 + j and the bottom position below it); the first
  // of them writes its norms and scales.
  constexpr int G = 16 / J;
  const int jl = lane16 / G;
  const bool lead = (lane16 & (G - 1)) == 0;
  int rc = 0;  // rounds since the start, mod CIRC (the circle's position)
  // Folds each scale into its column (w = d x), sets d = e = 1 and, at a
  // sweep's start, sums the exact squared norms; at a multiple of J rounds the
  // renaming is the identity, so slot j holds logical top / bottom j.
  auto rescale = [&](bool norms) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int it = active ? top_id(q0 + j, rc) : 0;
      const int ib = active ? bot_id(q0 + j, rc) : 0;
      const T dt = T(s_d[it]), db = T(s_d[ib]);
      T pa = 0, pb = 0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        tc[j][t] *= dt;
        bc[j][t] *= db;
        pa = fma(tc[j][t], tc[j][t], pa);
        pb = fma(bc[j][t], bc[j][t], pb);
      }
      if (norms) {
        pa = row_sum16(pa);
        pb = row_sum16(pb);
      }
      if (active && lane16 == 0) {
        s_d[it] = 1.0;
        s_e[it] = 1.0;
        s_d[ib] = 1.0;
        s_e[ib] = 1.0;
        if (norms) {
          s_norm[it] = double(pa);
          s_norm[ib] = double(pb);
        }
      }
    }
  };
  for (int q = threadIdx.x; q < 2 * H; q += kJacobiThreads) {
    s_d[q] = 1.0;
    s_e[q] = 1.0;
  }
  __syncthreads();
  for (;;) {
    for (int blk = 0; blk < 2 * nunits; ++blk) {
      // Exact norms at the start of every sweep; the scales are folded in
      // every kRescaleBlocks blocks, which bounds the growth of the stored
      // columns (at most sqrt(2) per rotation) to 2^(J kRescaleBlocks / 2).
      if (blk % kRescaleBlocks == 0) rescale(blk == 0);
      static_for<0, J>([&](auto RR) {
        constexpr int rr = decltype(RR)::value;
        {
          // gamma of the scaled columns x, y of each pair: the J lane partials
          // are summed over the row by a transposing reduction that leaves
          // pair j's sum in lanes j (16 / J) ..: across the row mirror (lanes
          // with bit 3 clear keep pairs 0, 1 and pass 2, 3), then the half
          // mirror (bit 2), then inside quads; the lanes of a quad end with
          // the same bits.
          T pg[J];
#pragma unroll
          for (int j = 0; j < J; ++j) {
            const T* x = tc[(j - rr) & M];
            const T* y = bc[(j + rr) & M];
            T a = 0;
#pragma unroll
            for (int t = 0; t < RPL; ++t) a = fma(x[t], y[t], a);
            pg[j] = a;
          }
          T sg;
          if constexpr (J == 4) {
            const bool b3 = (lane16 & 8) != 0, b2 = (lane16 & 4) != 0;
            const T k0 = b3 ? pg[2] : pg[0], s0 = b3 ? pg[0] : pg[2];
            const T k1 = b3 ? pg[3] : pg[1], s1 = b3 ? pg[1] : pg[3];
            const T h0 = k0 + dpp_move<0x140>(s0);  // row_mirror
            const T h1 = k1 + dpp_move<0x140>(s1);
            sg = (b2 ? h1 : h0) + dpp_move<0x141>(b2 ? h0 : h1);  // row_half_mirror
          } else if constexpr (J == 2) {
            const bool b3 = (lane16 & 8) != 0;
            sg = (b3 ? pg[1] : pg[0]) + dpp_move<0x140>(b3 ? pg[0] : pg[1]);
            sg += dpp_move<0x141>(sg);
          } else {
            sg = pg[0] + dpp_move<0x140>(pg[0]);
            sg += dpp_move<0x141>(sg);
          }
          sg += dpp_move<0x4e>(sg);  // quad_perm [2,3,0,1]
          sg += dpp_move<0xb1>(sg);  // quad_perm [1,0,3,2]
          // w_i = d_i x_i, w_j = d_j x_j, so the inner product of the
          // columns is d_i d_j (x_i . x_j); alpha and beta are the carried
          // squared norms of w_i, w_j.
          const int id_t = active ? top_id(q0 + jl, rc) : 0;
          const int id_b = active ? bot_id(q0 + jl, rc) : 0;
          const double al = s_norm[id_t], be = s_norm[id_b];
          const double di = s_d[id_t], dj = s_d[id_b];
          const double ei = s_e[id_t], ej = s_e[id_b];
          const double gam = double(sg) * di * dj;
          double cd, sd, td;
          const int flag = rotation_t<kRotNewton<T>>(al, be, gam, tol, cd, sd, td);
          if (lead) {
            my_rot += flag == 1;
            my_bad |= flag == 2;
          }
          // Scaled rotation as two shears, each an FMA in place:
          //   x_j' = x_j + b x_i,  b = t d_i / d_j,             d_j' = c d_j;
          //   x_i' = x_i - a x_j', a = t d_j / (d_i (1 + t^2)), d_i' = d_i / c;
          // then d_i' x_i' = c w_i - s w_j and d_j' x_j' = s w_i + c w_j (the
          // rotation that zeroes gamma).  The stored values of one column grow
          // by 1 / c <= sqrt(2) and those of the other shrink by c.  e = 1 / d is
          // carried too (1 / c = c (1 + t^2)).
          const double ic = cd * fma(td, td, 1.0);
          const T fb = T(td * di * ej);
          const T fa = T(td * dj * ei * cd * cd);
          if (active && lead && flag == 1) {
            s_norm[id_t] = fma(-td, gam, al);
            s_norm[id_b] = fma(td, gam, be);
            s_d[id_t] = ic * di;
            s_d[id_b] = cd * dj;
            s_e[id_t] = cd * ei;
            s_e[id_b] = ic * ej;
          }
          static_for<0, J>([&](auto JJ) {
            constexpr int j = decltype(JJ)::value;
            const T ax = row_bcast<j * G>(fa), bx = row_bcast<j * G>(fb);
            T* x = tc[(j - rr) & M];
            T* y = bc[(j + rr) & M];
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              y[t] = fma(bx, x[t], y[t]);
              x[t] = fma(-ax, y[t], x[t]);
            }
          });
          // Outgoing columns: logical top J-1 and bottom 0 (and unit 0's fixed top 0).
          T* ot = &s_x[0][0][unit][0] + par * PAR;
          T* ob = &s_x[0][1][unit][0] + par * PAR;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            ot[lane16 + 16 * t] = tc[(M - rr) & M][t];
            ob[lane16 + 16 * t] = bc[rr & M][t];
          }
          if (wave == 0) {
            T* fx = &s_fx[0][0] + par * SLOT;
            if (unit == 0) {
#pragma unroll
              for (int t = 0; t < RPL; ++t) fx[lane16 + 16 * t] = tc[(J - rr) & M][t];
            }
          }
        }
        __syncthreads();
        {
          // Incoming columns land in the register slots the outgoing ones left.
          const T* it = in_top + par * in_top_par;
          const T* ib = in_bot + par * PAR;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            tc[(M - rr) & M][t] = it[lane16 + 16 * t];
            bc[rr & M][t] = ib[lane16 + 16 * t];
          }
          if (J > 1 && wave == 0) {
            // Unit 0's top 1 takes its own former bottom 0.
            const T* b0 = &s_x[0][1][0][0] + par * PAR;
            const bool u0 = unit == 0;
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              const T v = b0[lane16 + 16 * t];
              tc[(J - rr) & M][t] = u0 ? v : tc[(J - rr) & M][t];
            }
          }
        }
        par ^= 1;
        rc = rc + 1 == CIRC ? 0 : rc + 1;
      });
    }
    // End of a sweep: converged if no pair rotated.
    const int sp = sw & 1;
    if (my_rot) atomicAdd(&s_rot[sp], my_rot);
    if (my_bad) s_bad = 1;
    my_rot = 0;
    __syncthreads();
    const bool done = s_rot[sp] == 0;
    const bool bad = s_bad != 0;
    if (threadIdx.x == 0) s_rot[sp ^ 1] = 0;
    ++sw;
    if (bad || done || sw >= max_sweeps) {
      converged = done && !bad;
      break;
    }
  }
  rescale(false);  // the columns of W themselves
  // The factors are formed from the registers: W never goes to memory.  The
  // norms, scales and exchange buffers are free from here on (s_sigma holds
  // the singular values, s_x the ranks and the staged output columns).
  __syncthreads();
  // After sw sweeps the circle has advanced sw * 2H = sw (mod CIRC) positions.
  const int rf = sw % CIRC;
  if (active) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      double pt = 0, pb = 0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        pt = fma(double(tc[j][t]), double(tc[j][t]), pt);
        pb = fma(double(bc[j][t]), double(bc[j][t]), pb);
      }
      pt = row_sum16(pt);
      pb = row_sum16(pb);
      const int cti = top_id(q0 + j, rf), cbi = bot_id(q0 + j, rf);
      if (lane16 == 0) {
        if (cti < nc) s_sigma[cti] = sqrt(pt);
        if (cbi < nc) s_sigma[cbi] = sqrt(pb);
      }
    }
  }
  __syncthreads();
  constexpr int kOrd = int(sizeof(s_order) / sizeof(int));
  static_assert(sizeof(s_x) >= 2 * kOrd * sizeof(int) + 128 * 16 * RPL * sizeof(T),
                "the exchange buffers stage at least 128 columns of 16 RPL rows");
  int* const s_rank = reinterpret_cast<int*>(&s_x[0][0][0][0]);
  rank_columns(nc, s_sigma, s_order, s_rank);
  __syncthreads();
  int cti[J], cbi[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    cti[j] = active ? top_id(q0 + j, rf) : nc;
    cbi[j] = active ? bot_id(q0 + j, rf) : nc;
  }
  // In s_x: ranks (kOrd ints), signs (kOrd ints), then the staged columns.
  emit_from_registers<T, J, RPL>(tc, bc, cti, cbi, d, slice, lane16, s_sigma, s_order, s_rank,
                                 s_rank + kOrd, reinterpret_cast<T*>(s_rank + 2 * kOrd),
                                 int((sizeof(s_x) - 2 * kOrd * sizeof(int)) / sizeof(T)), uhat,
                                 shat, vhat, us);
  if (threadIdx.x == 0) info[slice] = converged ? sw : -sw;
}

// The factor the register-resident kernel did not form, from A V = U Sigma:
// vhat_i = A^T u_i / sigma_i (n1 >= n2), or u_i = A vhat_i / sigma_i (n1 < n2),
// accumulated in FP64 from the coefficients.  In the second case the sign
// convention (largest |U| entry positive) is applied here to both columns,
// and U * sigma is written for the rebuild.  One workgroup per (slice, block
// of kRecCols columns), which reads the slice once for the block; columns with
// sigma_i at or below max(n1, n2) u sigma_1 come out zero.
constexpr int kRecCols = 4;  // recovered columns per workgroup
template <typename T>
__global__ __launch_bounds__(256) void recover_kernel(const T* __restrict__ ah, SvdDims d,
                                                      T* __restrict__ uhat,
                                                      const T* __restrict__ shat,
                                                      T* __restrict__ vhat, T* __restrict__ us) {
  const int k = d.k;
  const int slice = blockIdx.x;
  const int i0 = blockIdx.y * kRecCols;
  const int mr = d.mr, nc = d.nc;
  const T* A = ah + int64_t(slice) * d.n1 * d.n2;
  T* U = uhat + int64_t(slice) * d.n1 * k;
  T* Vo = vhat + int64_t(slice) * d.n2 * k;
  const T* src = d.trans ? Vo : U;  // the columns formed from W, mr entries
  T* dst = d.trans ? U : Vo;        // the columns recovered here, nc entries
  constexpr int kOut = kMaxSide / 256;
  // Dynamic LDS, sized by the launch: the kRecCols source columns (mr values
  // each), then (transposed slices only) the sign search of every column.
  extern __shared__ double s_dyn[];
  double* const s_src = s_dyn;  // [kRecCols][mr]
  double* const s_best = s_dyn + kRecCols * mr;  // [kRecCols][256]
  double* const s_val = s_best + kRecCols * 256;  // [kRecCols][256]
  int* const s_row = reinterpret_cast<int*>(s_val + kRecCols * 256);  // [kRecCols][256]
  // Columns of singular values at or below the numerical rank cut
  // max(n1, n2) u sigma_1 (the cut of the pseudo-inverse) are not recovered
  // (zero): A^T u_i / sigma_i would amplify the rounding of u_i beyond one.
  const double cut = double(mr) * Unit<T>::value * double(shat[int64_t(slice) * k]);
  double sg[kRecCols], inv[kRecCols];
#pragma unroll
  for (int c = 0; c < kRecCols; ++c) {
    const int i = i0 + c < k ? i0 + c : i0;
    sg[c] = double(shat[int64_t(slice) * k + i]);
    inv[c] = (i0 + c < k && sg[c] > cut) ? 1.0 / sg[c] : 0.0;
  }
  for (int t = threadIdx.x; t < mr; t += 256)
#pragma unroll
    for (int c = 0; c < kRecCols; ++c)
      s_src[c * mr + t] = i0 + c < k ? double(src[int64_t(t) * k + i0 + c]) : 0.0;
  __syncthreads();
  double out[kOut][kRecCols];
  double best[kRecCols], bval[kRecCols];
  int brow[kRecCols];
#pragma unroll
  for (int c = 0; c < kRecCols; ++c) {
    best[c] = -1.0;
    bval[c] = 0.0;
    brow[c] = 0x7fffffff;
  }
#pragma unroll
  for (int j = 0; j < kOut; ++j) {
    const int r = threadIdx.x + 256 * j;
    double acc[kRecCols] = {};
    if (r < nc) {
      // Each element of the slice is read once for all kRecCols columns.
      if (d.trans)
        for (int t = 0; t < mr; ++t) {
          const double a = double(A[int64_t(r) * d.n2 + t]);
#pragma unroll
          for (int c = 0; c < kRecCols; ++c) acc[c] = fma(a, s_src[c * mr + t], acc[c]);
        }
      else
        for (int t = 0; t < mr; ++t) {
          const double a = double(A[int64_t(t) * d.n2 + r]);
#pragma unroll
          for (int c = 0; c < kRecCols; ++c) acc[c] = fma(a, s_src[c * mr + t], acc[c]);
        }
#pragma unroll
      for (int c = 0; c < kRecCols; ++c) {
        acc[c] *= inv[c];
        if (fabs(acc[c]) > best[c]) {
          best[c] = fabs(acc[c]);
          brow[c] = r;
          bval[c] = acc[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kRecCols; ++c) out[j][c] = acc[c];
  }
  double sgn[kRecCols];
#pragma unroll
  for (int c = 0; c < kRecCols; ++c) sgn[c] = 1.0;
  if (d.trans) {
    // Largest |U| entry over each column, lowest row on ties.
#pragma unroll
    for (int c = 0; c < kRecCols; ++c) {
      s_best[c * 256 + threadIdx.x] = best[c];
      s_row[c * 256 + threadIdx.x] = brow[c];
      s_val[c * 256 + threadIdx.x] = bval[c];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const int o = threadIdx.x + w;
#pragma unroll
        for (int c = 0; c < kRecCols; ++c) {
          const int me = c * 256 + threadIdx.x, ot = c * 256 + o;
          if (s_best[ot] > s_best[me] || (s_best[ot] == s_best[me] && s_row[ot] < s_row[me])) {
            s_best[me] = s_best[ot];
            s_row[me] = s_row[ot];
            s_val[me] = s_val[ot];
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < kRecCols; ++c) sgn[c] = s_val[c * 256] < 0 ? -1.0 : 1.0;
  }
#pragma unroll
  for (int j = 0; j < kOut; ++j) {
    const int r = threadIdx.x + 256 * j;
    if (r < nc)
#pragma unroll
      for (int c = 0; c < kRecCols; ++c) {
        if (i0 + c >= k) continue;
        const T x = T(sgn[c] * out[j][c]);
        dst[int64_t(r) * k + i0 + c] = x;
        if (d.trans) us[int64_t(slice) * d.n1 * k + int64_t(r) * k + i0 + c] = T(x * T(sg[c]));
      }
  }
  if (d.trans)
#pragma unroll
    for (int c = 0; c < kRecCols; ++c)
      if (i0 + c < k && sgn[c] < 0)
        for (int t = threadIdx.x; t < mr; t += 256) Vo[int64_t(t) * k + i0 + c] = T(-s_src[c * mr + t]);
}

// Gram matrix G = X^T X (FP64) of one slice X (n x k row-major, k <= 64) for
// 256 threads: thread t accumulates entries e = t + 256 q (a = e / k, b = e % k)
// in acc[q]; rows are staged through LDS in blocks of kGramRows as FP64, so n
// is unbounded.
constexpr int kGramRows = 64;
template <typename T>
__device__ __forceinline__ void gram_k64(const T* __restrict__ X, int n, int k, double (&acc)[16],
                                         double* s_blk) {
  // Entry slots q < nq hold entries (the same for every thread: a uniform
  // branch), and each slot's (a, b) is fixed over the rows.
  const int nq = (k * k + 255) / 256;
  int ia[16], ib[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    acc[q] = 0;
    const int e = threadIdx.x + 256 * q;
    const bool in = e < k * k;
    ia[q] = in ? e / k : 0;
    ib[q] = in ? e - (e / k) * k : 0;
  }
  for (int r0 = 0; r0 < n; r0 += kGramRows) {
    const int rows = n - r0 < kGramRows ? n - r0 : kGramRows;
    __syncthreads();
    for (int e = threadIdx.x; e < rows * k; e += 256) s_blk[e] = double(X[int64_t(r0) * k + e]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (q < nq) {
        const double* xa = s_blk + ia[q];
        const double* xb = s_blk + ib[q];
        double s = acc[q];
        for (int r = 0; r < rows; ++r) s = fma(xa[r * k], xb[r * k], s);
        acc[q] = s;
      }
    }
  }
  // Entries past k * k stay exactly zero (they multiplied row 0's column 0
  // only in slots that are not used).
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (threadIdx.x + 256 * q >= k * k) acc[q] = 0;
}

// The same Gram matrix of a slice already in LDS as FP64 (n x k row-major).
__device__ __forceinline__ void gram_lds(const double* __restrict__ s_x, int n, int k,
                                         double (&acc)[16]) {
  const int nq = (k * k + 255) / 256;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    acc[q] = 0;
    const int e = threadIdx.x + 256 * q;
    if (q < nq && e < k * k) {
      const int a = e / k, b = e - a * k;
      double s = 0;
      for (int r = 0; r < n; ++r) s = fma(s_x[r * k + a], s_x[r * k + b], s);
      acc[q] = s;
    }
  }
}

// Largest |G_ab - delta_ab| over the columns a, b that are not identically
// zero (G_aa > 0), NaN-propagating; every thread of the 256 returns it.
// Columns that are zero belong to singular values at or below the numerical
// rank cut and are left out of the orthogonality measure.
__device__ __forceinline__ double gram_dev(const double* __restrict__ G, int k, double* red) {
  double worst = 0;
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int a = e / k, b = e - a * k;
    if (G[int64_t(a) * k + a] == 0.0 || G[int64_t(b) * k + b] == 0.0) continue;
    const double dev = fabs(G[e] - (a == b ? 1.0 : 0.0));
    worst = (dev > worst || dev != dev) ? dev : worst;
  }
  __syncthreads();
  red[threadIdx.x] = worst;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = red[threadIdx.x + w];
      const double m = red[threadIdx.x];
      red[threadIdx.x] = (o > m || o != o) ? o : m;
    }
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Newton-Schulz polish of the recovered factor X (n x k per slice, row-major):
// the polar iteration X <- X (3 I - X^T X) / 2 = X M, M = 1.5 I - 0.5 G, in
// FP64 from the stored values.  The recovery inherits the error of the
// Jacobi-formed factor amplified by sigma_1 / sigma_i, and each step squares
// the deviation from orthonormality (e -> ~0.75 e^2), so the loop stops when
// the deviation is at the rounding level of T (no step) or after the step
// taken from a deviation below sqrt(u_T) / 4, and takes at most kPolishSteps
// steps.  Zero columns (singular values at or below the numerical rank cut)
// stay zero: their rows and columns of G are zero, so M maps them to zero and
// adds nothing to the others.
constexpr int kPolishSteps = 4;

// Deviation thresholds of the polish for n rows of T: at or below t_done the
// factor is orthonormal to the rounding of T (storing a column in T moves the
// Gram entries by up to 2 u_T, and the FP64 Gram itself is accurate to about
// sqrt(n) u_64); from at or below t_last one more step reaches it.
template <typename T>
__host__ __device__ inline void polish_thresholds(int n, double& t_done, double& t_last) {
  const double u = Unit<T>::value;
  t_done = 4.0 * u + 4.0 * sqrt(double(n)) * Unit<double>::value;
  t_last = 0.25 * sqrt(u);
}

// k <= 64: one workgroup per slice, G and M in LDS.  When the slice fits
// (n k <= kPolishLds values) it is read into LDS once and every pass runs
// from there; otherwise the rows are streamed through LDS in blocks (each
// row's update reads only that row, so the blocks are updated in place).
constexpr int kPolishLds = 8192;
template <typename T>
__global__ __launch_bounds__(256) void polish_kernel(T* __restrict__ x, int n, int k) {
  __shared__ double s_m[64 * 64];
  __shared__ double s_x[kPolishLds];
  __shared__ double s_red[256];
  T* X = x + int64_t(blockIdx.x) * n * k;
  double t_done, t_last;
  polish_thresholds<T>(n, t_done, t_last);
  const bool whole = n * k <= kPolishLds;
  if (whole)
    for (int e = threadIdx.x; e < n * k; e += 256) s_x[e] = double(X[e]);
  for (int step = 0; step < kPolishSteps; ++step) {
    double acc[16];
    if (whole)
      gram_lds(s_x, n, k, acc);
    else
      gram_k64<T>(X, n, k, acc, s_x);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < k * k) s_m[e] = acc[q];
    }
    __syncthreads();
    const double dev = gram_dev(s_m, k, s_red);
    if (dev <= t_done) return;
    for (int e = threadIdx.x; e < k * k; e += 256) {
      const int a = e / k, b = e - a * k;
      s_m[e] = (a == b ? 1.5 : 0.0) - 0.5 * s_m[e];
    }
    // X[r][i] = sum_j X[r][j] M[j][i]; consecutive threads take consecutive i,
    // so M reads are conflict-free and X reads broadcast.
    if (whole) {
      constexpr int kPer = kPolishLds / 256;
      double nx[kPer];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = threadIdx.x + 256 * q;
        double a2 = 0;
        if (e < n * k) {
          const int r = e / k, i = e - r * k;
          const double* xr = s_x + r * k;
          for (int j = 0; j < k; ++j) a2 = fma(xr[j], s_m[j * k + i], a2);
        }
        nx[q] = a2;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < n * k) {
          const T v = T(nx[q]);
          X[e] = v;
          s_x[e] = double(v);  // the stored value, as the next pass reads it
        }
      }
    } else {
      for (int r0 = 0; r0 < n; r0 += kGramRows) {
        const int rows = n - r0 < kGramRows ? n - r0 : kGramRows;
        T* Xb = X + int64_t(r0) * k;
        __syncthreads();
        for (int e = threadIdx.x; e < rows * k; e += 256) s_x[e] = double(Xb[e]);
        __syncthreads();
        for (int e = threadIdx.x; e < rows * k; e += 256) {
          const int r = e / k, i = e - r * k;
          const double* xr = s_x + r * k;
          double a2 = 0;
          for (int j = 0; j < k; ++j) a2 = fma(xr[j], s_m[j * k + i], a2);
          Xb[e] = T(a2);
        }
      }
    }
    if (!(dev > t_last)) return;  // NaN: stop as well
  }
}

// Per-slice C = op(A) B with FP64 accumulation, a small helper GEMM of the
// polish and the orthogonality check for k > 64 (off the benchmark path).
// op(A) is m x kk: A stored kk x m (row-major) when TRA, m x kk otherwise; B
// is kk x n and C m x n, row-major; slices at strides sa, sb, sc.  A 64 x 64
// tile of C per workgroup (4 x 4 per thread), kk in chunks of 16 through LDS.
// Slices whose state is 1 are skipped.
template <typename TA, typename TB, typename TC, bool TRA>
__global__ __launch_bounds__(256) void small_gemm_kernel(const TA* __restrict__ a,
                                                         const TB* __restrict__ b,
                                                         TC* __restrict__ c, int m, int kk, int n,
                                                         int64_t sa, int64_t sb, int64_t sc,
                                                         const int* __restrict__ state) {
  const int slice = blockIdx.z;
  if (state != nullptr && state[slice] == 1) return;
  __shared__ double s_a[16][65];
  __shared__ double s_b[16][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const TA* A = a + slice * sa;
  const TB* B = b + slice * sb;
  TC* C = c + slice * sc;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;
  for (int k0 = 0; k0 < kk; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int kq, r;
      if (TRA) {
        kq = e >> 6;
        r = e & 63;
      } else {
        r = e >> 4;
        kq = e & 15;
      }
      const int gr = r0 + r, gk = k0 + kq;
      double v = 0;
      if (gr < m && gk < kk)
        v = TRA ? double(A[int64_t(gk) * m + gr]) : double(A[int64_t(gr) * kk + gk]);
      s_a[kq][r] = v;
    }
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int kq = e >> 6, cc = e & 63;
      const int gk = k0 + kq, gc = c0 + cc;
      s_b[kq][cc] = (gk < kk && gc < n) ? double(B[int64_t(gk) * n + gc]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = s_a[q][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = s_b[q][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty + 16 * i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = c0 + tx + 16 * j;
      if (r < m && cc < n) C[int64_t(r) * n + cc] = TC(acc[i][j]);
    }
  }
}

// k > 64 polish, one step over all slices: G (k x k, FP64, per slice) holds
// X^T X on entry.  state: 0 polishing, 2 the step formed here is the last, 1
// done (the later kernels of the step skip the slice).  Turns G into
// M = 1.5 I - 0.5 G, or marks the slice done.
template <typename T>
__global__ __launch_bounds__(256) void ns_form_kernel(double* __restrict__ g, int n, int k,
                                                      int* __restrict__ state) {
  __shared__ double s_red[256];
  const int slice = blockIdx.x;
  const int st = state[slice];
  if (st != 0) {
    if (st == 2 && threadIdx.x == 0) state[slice] = 1;
    return;
  }
  double* G = g + int64_t(slice) * k * k;
  double t_done, t_last;
  polish_thresholds<T>(n, t_done, t_last);
  const double dev = gram_dev(G, k, s_red);
  if (dev <= t_done) {
    if (threadIdx.x == 0) state[slice] = 1;
    return;
  }
  for (int64_t e = threadIdx.x; e < int64_t(k) * k; e += 256) {
    const int64_t a = e / k, b = e - a * k;
    G[e] = (a == b ? 1.5 : 0.0) - 0.5 * G[e];
  }
  if (threadIdx.x == 0 && !(dev > t_last)) state[slice] = 2;
}

// X <- Y for the slices still polishing (state != 1).
template <typename T>
__global__ __launch_bounds__(256) void ns_copy_kernel(const T* __restrict__ y, T* __restrict__ x,
                                                      int64_t per, const int* __restrict__ state) {
  const int slice = blockIdx.y;
  if (state[slice] == 1) return;
  const T* ys = y + slice * per;
  T* xs = x + slice * per;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < per; e += int64_t(gridDim.x) * 256)
    xs[e] = ys[e];
}

// Orthogonality of one slice from its Gram matrix in memory (k > 64).
__global__ __launch_bounds__(256) void gram_dev_kernel(const double* __restrict__ g, int k,
                                                       double* __restrict__ part) {
  __shared__ double s_red[256];
  const double dev = gram_dev(g + int64_t(blockIdx.x) * k * k, k, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = dev;
}

// max |X^T X - I| over the k x k Gram matrix of one slice of X (n x k,
// row-major, k <= 64), FP64, zero columns left out; both factors in one
// launch (workgroups [0, nsl) take X0 = U, [nsl, 2 nsl) X1 = V), part[f nsl +
// slice].
template <typename T>
__global__ __launch_bounds__(256) void orth_kernel(const T* __restrict__ x0,
                                                   const T* __restrict__ x1, int n0, int n1,
                                                   int k, int nsl, double* __restrict__ part) {
  __shared__ double s_g[64 * 64];
  __shared__ double s_blk[kGramRows * 64];
  __shared__ double s_red[256];
  const int f = int(blockIdx.x) >= nsl ? 1 : 0;
  const int slice = int(blockIdx.x) - f * nsl;
  const T* x = f ? x1 : x0;
  const int n = f ? n1 : n0;
  double acc[16];
  gram_k64<T>(x + int64_t(slice) * n * k, n, k, acc, s_blk);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (e < k * k) s_g[e] = acc[q];
  }
  __syncthreads();
  const double dev = gram_dev(s_g, k, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = dev;
}

// out[b] = max over part[b n, (b + 1) n), NaN-propagating; one workgroup per b.
__global__ __launch_bounds__(256) void max_reduce_kernel(const double* __restrict__ part, int64_t n,
                                                         double* __restrict__ out) {
  part += int64_t(blockIdx.x) * n;
  double worst = 0;
  for (int64_t e = threadIdx.x; e < n; e += 256) {
    const double v = part[e];
    worst = (v > worst || v != v) ? v : worst;
  }
  __shared__ double red[256];
  red[threadIdx.x] = worst;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = red[threadIdx.x + s];
      const double m = red[threadIdx.x];
      red[threadIdx.x] = (o > m || o != o) ? o : m;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Which Jacobi kernel a call takes.  Register-resident kernel when the
// columns fit (each of up to 32 units of 16 lanes owns J slots, J the
// smallest power of two with 32 * J >= nc_pad / 2, rpl rows per lane) and
// there are enough slices to occupy the chip with one workgroup each (64 or
// more), or the slices are too narrow (under 64 columns, at most two block
// pairs) to spread; the block kernel, which spreads a slice over several
// workgroups, otherwise.
// Slice count from which one workgroup per slice beats the block kernel
// (measured: 6 slices of 256 x 192 run 1.8x faster in the block kernel, 96
// take the same time both ways, 192 of 256 x 256 run 1.4x faster in the
// register kernel).
constexpr int64_t kRegMinSlices = 64;

struct JacobiChoice {
  bool reg;
  int J, nunits, rpl;
  BjShape bj;
};

inline JacobiChoice choose_jacobi(int mr, int nc, size_t es, int64_t nsl) {
  JacobiChoice c{};
  int ncp = nc + (nc & 1);
  if (ncp < 2) ncp = 2;
  const int half = ncp / 2;
  c.J = 1;
  while (c.J * kUnits < half) c.J *= 2;
  c.nunits = (half + c.J - 1) / c.J;
  c.rpl = 1;
  while (c.rpl * 16 < mr) c.rpl *= 2;
  c.reg = c.rpl <= 16 && c.J <= 4 && (es == 4 || (c.rpl <= 8 && c.J * c.rpl <= 16)) &&
          (nsl >= kRegMinSlices || nc < 64);
  c.bj = bj_shape(mr, nc);
  return c;
}

struct SvdPlan {
  size_t ah, w, us, ctl, part, gram, y, state, total;
};

// p coefficient slices are lifted; the first nsl of them are decomposed
// (nsl = p for w-svd, 2 p / 2^L for sp-w-svd).  With polish (w-svd, not the
// pseudo-inverse) and k > 64 the plan also holds the FP64 Gram matrices and
// the update buffer of the Newton-Schulz steps and of the orthogonality check.
inline SvdPlan plan_svd(int64_t n1, int64_t n2, int64_t p, int64_t nsl, int k, size_t es,
                        bool polish) {
  const int64_t mr = n1 > n2 ? n1 : n2;
  const int64_t nc = n1 > n2 ? n2 : n1;
  const JacobiChoice jc = choose_jacobi(int(mr), int(nc), es, nsl);
  // Columns of W in memory: the register kernel keeps W in registers.
  const int64_t ncw = jc.reg ? 0 : int64_t(jc.bj.nbp) * jc.bj.B;
  SvdPlan pl{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  pl.ah = take(size_t(p * n1 * n2) * es);  // coefficients, later the rebuilt ones
  pl.w = take(size_t(nsl * ncw * mr) * es);
  pl.us = take(size_t(nsl * n1 * k) * es);
  pl.ctl = take(size_t(nsl) * sizeof(BjCtl));
  pl.part = take(size_t(nsl) * 2 * sizeof(double));
  const bool big = polish && k > 64;
  pl.gram = take(big ? size_t(nsl) * k * k * sizeof(double) : 0);
  pl.y = take(big ? size_t(nsl * (n1 > n2 ? n1 : n2)) * k * es : 0);
  pl.state = take(size_t(nsl) * sizeof(int));
  pl.total = off + 256;
  return pl;
}

// Zeroes x[0, n) with plain vector stores (no memset node, so the call
// sequence stays capturable).
template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T* __restrict__ x, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    x[i] = T(0);
}

template <typename T>
hipError_t run_svd(const T* a, int64_t n1, int64_t n2, int64_t p, int L, int k, bool sparse,
                   T* uhat, T* shat, T* vhat, T* ak, int max_sweeps, int32_t* info,
                   double* orth_err, void* ws, hipStream_t s, bool second_factor = true,
                   hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr) {
  // sp-w-svd decomposes only s_L and d_L, the leading 2 p / 2^L coefficient
  // slices; the finer details are dropped (zero) in the rebuild.
  const int64_t nsl = sparse ? 2 * (p >> L) : p;
  const SvdPlan pl = plan_svd(n1, n2, p, nsl, k, sizeof(T), second_factor);
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
  T* ah = reinterpret_cast<T*>(base + pl.ah);
  T* w = reinterpret_cast<T*>(base + pl.w);
  T* us = reinterpret_cast<T*>(base + pl.us);
  BjCtl* ctl = reinterpret_cast<BjCtl*>(base + pl.ctl);
  double* part = reinterpret_cast<double*>(base + pl.part);
  double* gram = reinterpret_cast<double*>(base + pl.gram);
  T* ybuf = reinterpret_cast<T*>(base + pl.y);
  int* state = reinterpret_cast<int*>(base + pl.state);

  hipError_t e;
  if constexpr (sizeof(T) == 8)
    e = launch_lift_f64(LiftKind::kForward, reinterpret_cast<const double*>(a),
                        reinterpret_cast<double*>(ah), n1 * n2, p, L, s);
  else
    e = launch_lift_f32(LiftKind::kForward, reinterpret_cast<const float*>(a),
                        reinterpret_cast<float*>(ah), n1 * n2, p, L, s);
  if (e != hipSuccess) return e;

  SvdDims d{};
  d.n1 = int(n1);
  d.n2 = int(n2);
  d.mr = int(n1 > n2 ? n1 : n2);
  d.nc = int(n1 > n2 ? n2 : n1);
  d.ncp = d.nc + (d.nc & 1);
  if (d.ncp < 2) d.ncp = 2;
  d.k = k;
  d.trans = n1 < n2 ? 1 : 0;
  if (max_sweeps <= 0) max_sweeps = sizeof(T) == 8 ? 30 : 20;

  const JacobiChoice jc = choose_jacobi(d.mr, d.nc, sizeof(T), nsl);
  if (ev_begin != nullptr) {
    e = hipEventRecord(ev_begin, s);
    if (e != hipSuccess) return e;
  }
  if (jc.reg) {
    const dim3 grid{unsigned(nsl)};
    const dim3 block{unsigned(kJacobiThreads)};
    const int J = jc.J, rpl = jc.rpl, nunits = jc.nunits;
#define WP_JREG(JJ, RR)                                                                        \
  if (J == JJ && rpl == RR)                                                                    \
    hipLaunchKernelGGL((jacobi_reg_kernel<T, JJ, RR>), grid, block, 0, s, ah, d, nunits,        \
                       max_sweeps, uhat, shat, vhat, us, info);
    WP_JREG(1, 1) WP_JREG(1, 2) WP_JREG(1, 4) WP_JREG(1, 8)
    WP_JREG(2, 1) WP_JREG(2, 2) WP_JREG(2, 4) WP_JREG(2, 8)
    WP_JREG(4, 1) WP_JREG(4, 2) WP_JREG(4, 4)
    if constexpr (sizeof(T) == 4) {
      WP_JREG(1, 16) WP_JREG(2, 16) WP_JREG(4, 8) WP_JREG(4, 16)
    }
#undef WP_JREG
  } else {
    const BjShape b = jc.bj;
    const int ncb = b.nbp * b.B;
    const int64_t nctl = nsl * int64_t(sizeof(BjCtl) / sizeof(int));
    hipLaunchKernelGGL((zero_kernel<int>), dim3(unsigned((nctl + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<int*>(ctl), nctl);
    hipLaunchKernelGGL((bj_init_kernel<T>),
                       dim3(unsigned((d.mr + 31) / 32), unsigned((ncb + 31) / 32), unsigned(nsl)),
                       dim3(256), 0, s, ah, w, d, ncb, ctl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double tol = sqrt(double(d.mr)) * Unit<T>::value;
    const dim3 rgrid{unsigned(b.nbp / 2), unsigned(nsl)};
    for (int sw = 0; sw < max_sweeps; ++sw) {
      for (int r = 0; r + 1 < b.nbp; ++r) {
        bool launched = false;
#define WP_BJ(BB, RR)                                                                          \
  if (b.B == BB && b.rpl == RR) {                                                              \
    hipLaunchKernelGGL((bj_round_kernel<T, BB, RR>), rgrid, dim3(kBjThreads), 0, s, w, d.mr,    \
                       b.nbp, r, ctl, tol);                                                    \
    launched = true;                                                                           \
  }
        WP_BJ(16, 4) WP_BJ(16, 8) WP_BJ(16, 12) WP_BJ(16, 16)
        WP_BJ(16, 20) WP_BJ(16, 24) WP_BJ(16, 28) WP_BJ(16, 32)
        WP_BJ(8, 20) WP_BJ(8, 24) WP_BJ(8, 28) WP_BJ(8, 32)
#undef WP_BJ
        if (!launched) return hipErrorInvalidValue;  // shape outside the instantiated set
      }
      hipLaunchKernelGGL(bj_sweep_end_kernel, dim3(unsigned((nsl + 255) / 256)), dim3(256), 0, s,
                         ctl, int(nsl), max_sweeps);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((bj_emit_kernel<T>), dim3(unsigned(nsl)), dim3(kJacobiThreads), 0, s, w, d,
                       ncb, ctl, uhat, shat, vhat, us, info);
  }
  e = hipGetLastError();
  if (e == hipSuccess && ev_end != nullptr) e = hipEventRecord(ev_end, s);
  if (e != hipSuccess || !second_factor) return e;
  {
    // LDS sized to the slice (not to the largest one): more workgroups per CU.
    const size_t lds = size_t(kRecCols) * d.mr * sizeof(double) +
                       (d.trans ? size_t(kRecCols) * 256 * (2 * sizeof(double) + sizeof(int)) : 0);
    if (lds > 65536) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(recover_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((recover_kernel<T>),
                       dim3(unsigned(nsl), unsigned((k + kRecCols - 1) / kRecCols)), dim3(256), lds,
                       s, ah, d, uhat, shat, vhat, us);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  if (ak != nullptr) {
    // Rebuild Chat = (U sigma) V^T per slice (a face-product with inner size k),
    // reusing the coefficient region, then W^{-1}.
    if (nsl < p) {
      const int64_t tail = (p - nsl) * n1 * n2;
      const int64_t want = (tail + 255) / 256;
      const int64_t blocks = want < 8192 ? want : 8192;
      hipLaunchKernelGGL((zero_kernel<T>), dim3(unsigned(blocks)), dim3(256), 0, s,
                         ah + nsl * n1 * n2, tail);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if constexpr (sizeof(T) == 8) {
      e = launch_face_f64(reinterpret_cast<const double*>(us), reinterpret_cast<const double*>(vhat),
                          reinterpret_cast<double*>(ah), n1, k, n2, nsl, false, true, s);
      if (e == hipSuccess)
        e = launch_lift_f64(LiftKind::kInverse, reinterpret_cast<const double*>(ah),
                            reinterpret_cast<double*>(ak), n1 * n2, p, L, s);
    } else {
      e = launch_face_f32(reinterpret_cast<const float*>(us), reinterpret_cast<const float*>(vhat),
                          reinterpret_cast<float*>(ah), n1, k, n2, nsl, false, true, s);
      if (e == hipSuccess)
        e = launch_lift_f32(LiftKind::kInverse, reinterpret_cast<const float*>(ah),
                            reinterpret_cast<float*>(ak), n1 * n2, p, L, s);
    }
    if (e != hipSuccess) return e;
  }

  {
    // Orthonormalise the recovered factor (after the rebuild, which uses the
    // recovered columns as they are: their product with U is the exact rank-k
    // projection U U^T A).
    T* xr = d.trans ? uhat : vhat;
    const int nr = int(d.trans ? n1 : n2);
    if (k <= 64) {
      hipLaunchKernelGGL((polish_kernel<T>), dim3(unsigned(nsl)), dim3(256), 0, s, xr, nr, k);
    } else {
      hipLaunchKernelGGL((zero_kernel<int>), dim3(unsigned((nsl + 255) / 256)), dim3(256), 0, s,
                         state, nsl);
      const unsigned kt = unsigned((k + 63) / 64);
      const dim3 ggram{kt, kt, unsigned(nsl)};
      const dim3 gapply{kt, unsigned((nr + 63) / 64), unsigned(nsl)};
      const int64_t per = int64_t(nr) * k;
      const int64_t cb = (per + 255) / 256;
      const dim3 gcopy{unsigned(cb < 64 ? cb : 64), unsigned(nsl)};
      for (int step = 0; step < kPolishSteps; ++step) {
        hipLaunchKernelGGL((small_gemm_kernel<T, T, double, true>), ggram, dim3(256), 0, s, xr, xr,
                           gram, k, nr, k, per, per, int64_t(k) * k, state);
        hipLaunchKernelGGL((ns_form_kernel<T>), dim3(unsigned(nsl)), dim3(256), 0, s, gram, nr, k,
                           state);
        hipLaunchKernelGGL((small_gemm_kernel<T, double, T, false>), gapply, dim3(256), 0, s, xr,
                           gram, ybuf, nr, k, k, per, int64_t(k) * k, per, state);
        hipLaunchKernelGGL((ns_copy_kernel<T>), gcopy, dim3(256), 0, s, ybuf, xr, per, state);
      }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }

  if (orth_err != nullptr) {
    const T* fac[2] = {uhat, vhat};
    const int rows[2] = {int(n1), int(n2)};
    if (k <= 64) {
      hipLaunchKernelGGL((orth_kernel<T>), dim3(unsigned(2 * nsl)), dim3(256), 0, s, uhat, vhat,
                         int(n1), int(n2), k, int(nsl), part);
    } else {
      for (int f = 0; f < 2; ++f) {
        const unsigned kt = unsigned((k + 63) / 64);
        const int64_t per = int64_t(rows[f]) * k;
        hipLaunchKernelGGL((small_gemm_kernel<T, T, double, true>), dim3(kt, kt, unsigned(nsl)),
                           dim3(256), 0, s, fac[f], fac[f], gram, k, rows[f], k, per, per,
                           int64_t(k) * k, static_cast<const int*>(nullptr));
        hipLaunchKernelGGL(gram_dev_kernel, dim3(unsigned(nsl)), dim3(256), 0, s, gram, k,
                           part + f * nsl);
      }
    }
    hipLaunchKernelGGL(max_reduce_kernel, dim3(2), dim3(256), 0, s, part, nsl, orth_err);
    e = hipGetLastError();
  }
  return e;
}

// Pseudo-inverse of sigma applied to the columns of vhat (n2 x k per slice):
// column i is scaled by 1 / sigma_i when sigma_i > rtol * sigma_max, else
// zeroed (Def. 2.6 per coefficient slice; sigma is sorted, sigma_max first).
// x_i <- x_i / sigma_i^2 for sigma_i > rtol * sigma_0, else 0, for the k
// columns of each slice of x (rows x k); grid (x, nsl).
template <typename T>
__global__ __launch_bounds__(256) void pinv_scale_kernel(T* __restrict__ x,
                                                         const T* __restrict__ sh, int rows, int k,
                                                         double rtol) {
  const int64_t slice = blockIdx.y;
  const T* sg = sh + slice * k;
  const double cut = rtol * double(sg[0]);
  T* xs = x + slice * rows * k;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < int64_t(rows) * k;
       e += int64_t(gridDim.x) * 256) {
    const double si = double(sg[e % k]);
    const double inv = si > cut ? 1.0 / si : 0.0;
    xs[e] = T(double(xs[e]) * inv * inv);
  }
}

struct PinvPlan {
  size_t svd, uh, sh, vh, ph, total;
};

inline PinvPlan plan_pinv(int64_t n1, int64_t n2, int64_t p, int64_t nsl, size_t es) {
  const int64_t k = n1 < n2 ? n1 : n2;
  PinvPlan pl{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  const SvdPlan sp = plan_svd(n1, n2, p, nsl, int(k), es, false);
  pl.svd = take(sp.total);
  pl.uh = take(size_t(nsl * n1 * k) * es);
  pl.sh = take(size_t(nsl * k) * es);
  pl.vh = take(size_t(nsl * n2 * k) * es);
  pl.ph = take(size_t(p * n2 * n1) * es);
  pl.total = off + 256;
  return pl;
}

// A^+ = W^{-1}( P_c ) over the coefficient slices c (all p, or only s_L and
// d_L when sparse; the rest of the coefficients are zero).  Per slice A_c the
// Jacobi gives the factor F formed by W and sigma; with the cut values
// dropped, P_c = V Sigma^+ U^T is
//   A_c^T U Sigma^-2 U^T = (A_c^T F) (F Sigma^-2)^T      when n1 >= n2 (F = U),
//   V Sigma^-2 V^T A_c^T = (F Sigma^-2) (A_c F)^T        when n1 < n2 (F = V),
// two face-products on the matrix cores, with no recovered factor.  Both
// forms are exact for any F that spans the kept space.
template <typename T>
hipError_t run_pinv(const T* a, T* out, int64_t n1, int64_t n2, int64_t p, int L, bool sparse,
                    double rtol, int32_t* info, void* ws, hipStream_t s) {
  const int64_t k = n1 < n2 ? n1 : n2;
  const int64_t nsl = sparse ? 2 * (p >> L) : p;
  const PinvPlan pl = plan_pinv(n1, n2, p, nsl, sizeof(T));
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
  T* uh = reinterpret_cast<T*>(base + pl.uh);
  T* sh = reinterpret_cast<T*>(base + pl.sh);
  T* vh = reinterpret_cast<T*>(base + pl.vh);
  T* ph = reinterpret_cast<T*>(base + pl.ph);
  // The coefficient slices, lifted by run_svd into its own workspace region.
  const T* ah = reinterpret_cast<const T*>(base + pl.svd +
                                           plan_svd(n1, n2, p, nsl, int(k), sizeof(T), false).ah);
  hipError_t e = run_svd<T>(a, n1, n2, p, L, int(k), sparse, uh, sh, vh, static_cast<T*>(nullptr),
                            0, info, nullptr, base + pl.svd, s, /*second_factor=*/false);
  if (e != hipSuccess) return e;
  const bool trans = n1 < n2;
  // M = A^T U into vh (n2 x k), or A V into uh (n1 x k).
  if constexpr (sizeof(T) == 8) {
    e = trans ? launch_face_f64(reinterpret_cast<const double*>(ah),
                                reinterpret_cast<const double*>(vh), reinterpret_cast<double*>(uh),
                                n1, n2, k, nsl, false, false, s)
              : launch_face_f64(reinterpret_cast<const double*>(ah),
                                reinterpret_cast<const double*>(uh), reinterpret_cast<double*>(vh),
                                n2, n1, k, nsl, true, false, s);
  } else {
    e = trans ? launch_face_f32(reinterpret_cast<const float*>(ah),
                                reinterpret_cast<const float*>(vh), reinterpret_cast<float*>(uh),
                                n1, n2, k, nsl, false, false, s)
              : launch_face_f32(reinterpret_cast<const float*>(ah),
                                reinterpret_cast<const float*>(uh), reinterpret_cast<float*>(vh),
                                n2, n1, k, nsl, true, false, s);
  }
  if (e != hipSuccess) return e;
  // F Sigma^-2 in place (F = uh or vh).
  const int64_t rows = trans ? n2 : n1;
  const int64_t want = (rows * k + 255) / 256;
  hipLaunchKernelGGL((pinv_scale_kernel<T>), dim3(unsigned(want < 64 ? want : 64), unsigned(nsl)),
                     dim3(256), 0, s, trans ? vh : uh, sh, int(rows), int(k), rtol);
  if (nsl < p) {
    const int64_t tail = (p - nsl) * n2 * n1;
    const int64_t wt = (tail + 255) / 256;
    hipLaunchKernelGGL((zero_kernel<T>), dim3(unsigned(wt < 8192 ? wt : 8192)), dim3(256), 0, s,
                       ph + nsl * n2 * n1, tail);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // P = vh uh^T (n2 x n1), then W^{-1}.
  if constexpr (sizeof(T) == 8) {
    e = launch_face_f64(reinterpret_cast<const double*>(vh), reinterpret_cast<const double*>(uh),
                        reinterpret_cast<double*>(ph), n2, k, n1, nsl, false, true, s);
    if (e == hipSuccess)
      e = launch_lift_f64(LiftKind::kInverse, reinterpret_cast<const double*>(ph),
                          reinterpret_cast<double*>(out), n2 * n1, p, L, s);
  } else {
    e = launch_face_f32(reinterpret_cast<const float*>(vh), reinterpret_cast<const float*>(uh),
                        reinterpret_cast<float*>(ph), n2, k, n1, nsl, false, true, s);
    if (e == hipSuccess)
      e = launch_lift_f32(LiftKind::kInverse, reinterpret_cast<const float*>(ph),
                          reinterpret_cast<float*>(out), n2 * n1, p, L, s);
  }
  return e;
}

}  // namespace

size_t pinv_workspace_bytes(int64_t n1, int64_t n2, int64_t p, int L, bool sparse, int dtype) {
  return plan_pinv(n1, n2, p, sparse ? 2 * (p >> L) : p, dtype == 0 ? 8 : 4).total;
}

hipError_t launch_pinv(const void* a, void* out, int64_t n1, int64_t n2, int64_t p, int L,
                       bool sparse, double rtol, int32_t* info, int dtype, void* ws, hipStream_t s) {
  if (dtype == 0)
    return run_pinv<double>(static_cast<const double*>(a), static_cast<double*>(out), n1, n2, p, L,
                            sparse, rtol, info, ws, s);
  return run_pinv<float>(static_cast<const float*>(a), static_cast<float*>(out), n1, n2, p, L,
                         sparse, rtol, info, ws, s);
}

size_t svd_workspace_bytes(int64_t n1, int64_t n2, int64_t p, int L, int k, bool sparse,
                           int dtype) {
  return plan_svd(n1, n2, p, sparse ? 2 * (p >> L) : p, k, dtype == 0 ? 8 : 4, true).total;
}

hipError_t launch_svd(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k, bool sparse,
                      void* uhat, void* shat, void* vhat, void* ak, int max_sweeps, int32_t* info,
                      double* orth_err, int dtype, void* ws, hipStream_t s, hipEvent_t ev_begin,
                      hipEvent_t ev_end) {
  if (dtype == 0)
    return run_svd<double>(static_cast<const double*>(a), n1, n2, p, L, k, sparse,
                           static_cast<double*>(uhat),
                           static_cast<double*>(shat), static_cast<double*>(vhat),
                           static_cast<double*>(ak), max_sweeps, info, orth_err, ws, s, true,
                           ev_begin, ev_end);
  return run_svd<float>(static_cast<const float*>(a), n1, n2, p, L, k, sparse,
                        static_cast<float*>(uhat),
                        static_cast<float*>(shat), static_cast<float*>(vhat), static_cast<float*>(ak),
                        max_sweeps, info, orth_err, ws, s, true, ev_begin, ev_end);
}

}  // namespace wp
