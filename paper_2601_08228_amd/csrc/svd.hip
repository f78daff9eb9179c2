// w-svd (Alg. 2, Thm 2.5) for gfx950: per-coefficient-slice truncated SVD by
// one-sided (Hestenes) Jacobi, rank-k rebuild on the face-product GEMM, and
// the inverse lifting.
//
// Jacobi: one workgroup owns one coefficient slice.  The slice is copied into
// a column-major working matrix W (the slice itself when n1 >= n2, its
// transpose otherwise, so that W has mr = max(n1, n2) rows and nc = min(n1, n2)
// columns) and V starts as the identity.  A sweep visits every column pair
// once, in nc_pad - 1 rounds of nc_pad/2 disjoint pairs (round-robin
// tournament, one dummy column when nc is odd).  Each wavefront takes a batch
// of pairs of the round, issues all their column loads at once, forms
// alpha = |w_i|^2, beta = |w_j|^2, gamma = w_i.w_j in FP64 with wavefront
// reductions, and applies the rotation (angle in FP64) to W and V.  A pair is
// rotated when |gamma| > tol * sqrt(alpha * beta), tol = sqrt(mr) * unit
// roundoff of the data type; the slice has converged after a sweep with no
// rotation.  Columns live in the workspace, so they stay in the L2/MALL.
//
// Afterwards sigma_i = |w_i| (FP64), the columns are ranked by decreasing
// sigma (ties by index), the k leading ones are normalised into U, signs are
// fixed so that each U column's largest-magnitude entry is positive, and
// U * sigma is written for the rebuild.

#include "wp_internal.h"

namespace wp {
namespace {

constexpr int kJacobiWaves = 8;
constexpr int kJacobiThreads = 64 * kJacobiWaves;
constexpr int kPairBatch = 4;

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

// RPL: rows per lane (mr <= 64 * RPL).
template <typename T, int RPL>
__global__ __launch_bounds__(kJacobiThreads) void jacobi_kernel(
    const T* __restrict__ ah, T* __restrict__ wbuf, T* __restrict__ vbuf, SvdDims d,
    int max_sweeps, T* __restrict__ uhat, T* __restrict__ shat, T* __restrict__ vhat,
    T* __restrict__ us, int32_t* __restrict__ info) {
  const int slice = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int mr = d.mr, nc = d.nc, ncp = d.ncp;
  const T* a = ah + int64_t(slice) * d.n1 * d.n2;
  T* W = wbuf + int64_t(slice) * nc * mr;   // column c at W + c*mr
  T* V = vbuf + int64_t(slice) * nc * nc;   // column c at V + c*nc

  __shared__ int s_rot;
  __shared__ int s_bad;
  __shared__ double s_sigma[1024];
  __shared__ int s_order[1024];

  // ---- copy the slice into column-major W, V = I ---------------------------
  for (int64_t e = threadIdx.x; e < int64_t(mr) * nc; e += kJacobiThreads) {
    const int c = int(e / mr), r = int(e % mr);
    // W[r][c]: slice entry (r, c) if not transposed, (c, r) otherwise.
    W[e] = d.trans ? a[int64_t(c) * d.n2 + r] : a[int64_t(r) * d.n2 + c];
  }
  for (int64_t e = threadIdx.x; e < int64_t(nc) * nc; e += kJacobiThreads) {
    const int c = int(e / nc), r = int(e % nc);
    V[e] = T(r == c ? 1 : 0);
  }
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();

  const double tol = sqrt(double(mr)) * Unit<T>::value;
  const int npairs = ncp / 2;
  int sweeps = 0;
  bool converged = false;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (threadIdx.x == 0) s_rot = 0;
    __syncthreads();
    int my_rot = 0;
    for (int r = 0; r < ncp - 1; ++r) {
      for (int q0 = wave * kPairBatch; q0 < npairs; q0 += kJacobiWaves * kPairBatch) {
        int pi[kPairBatch], pj[kPairBatch];
        bool live[kPairBatch];
        T wi[kPairBatch][RPL], wj[kPairBatch][RPL], vi[kPairBatch][RPL], vj[kPairBatch][RPL];
#pragma unroll
        for (int b = 0; b < kPairBatch; ++b) {
          const int q = q0 + b;
          int i = 0, j = 0;
          if (q < npairs) rr_pair(ncp, r, q, i, j);
          live[b] = (q < npairs) && i < nc && j < nc;  // skip the dummy column
          pi[b] = i;
          pj[b] = j;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const int row = lane + 64 * t;
            const bool okw = live[b] && row < mr;
            const bool okv = live[b] && row < nc;
            wi[b][t] = okw ? W[int64_t(i) * mr + row] : T(0);
            wj[b][t] = okw ? W[int64_t(j) * mr + row] : T(0);
            vi[b][t] = okv ? V[int64_t(i) * nc + row] : T(0);
            vj[b][t] = okv ? V[int64_t(j) * nc + row] : T(0);
          }
        }
#pragma unroll
        for (int b = 0; b < kPairBatch; ++b) {
          double al = 0, be = 0, ga = 0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const double x = double(wi[b][t]), y = double(wj[b][t]);
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
          al = wave_sum(al);
          be = wave_sum(be);
          ga = wave_sum(ga);
          if (!live[b]) continue;
          if (!(isfinite(al) && isfinite(be) && isfinite(ga))) {
            if (lane == 0) s_bad = 1;
            continue;
          }
          if (!(fabs(ga) > tol * sqrt(al * be))) continue;
          ++my_rot;
          // Rotation that zeroes the (i, j) inner product (Rutishauser's form).
          const double zeta = (be - al) / (2.0 * ga);
          const double t = fabs(zeta) > 1e150 ? 0.5 / zeta
                                              : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
#pragma unroll
          for (int tt = 0; tt < RPL; ++tt) {
            const int row = lane + 64 * tt;
            const double x = double(wi[b][tt]), y = double(wj[b][tt]);
            if (row < mr) {
              W[int64_t(pi[b]) * mr + row] = T(c * x - s * y);
              W[int64_t(pj[b]) * mr + row] = T(s * x + c * y);
            }
            const double u = double(vi[b][tt]), v = double(vj[b][tt]);
            if (row < nc) {
              V[int64_t(pi[b]) * nc + row] = T(c * u - s * v);
              V[int64_t(pj[b]) * nc + row] = T(s * u + c * v);
            }
          }
        }
      }
      __syncthreads();  // the next round reads columns written in this one
    }
    if (lane == 0 && my_rot) atomicAdd(&s_rot, my_rot);
    __syncthreads();
    sweeps = sw + 1;
    const bool done = (s_rot == 0);
    const bool bad = (s_bad != 0);
    __syncthreads();
    if (bad) break;
    if (done) {
      converged = true;
      break;
    }
  }

  // ---- singular values, ordering ----------------------------------------------
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
  // Rank by a strict total order: larger sigma first, NaN after every number,
  // ties (and NaNs) by column index; the ranks are therefore a permutation.
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
  }
  __syncthreads();

  // ---- outputs: k leading triplets ----------------------------------------------
  // U column i has n1 entries, V column i has n2 entries.  Without transposition
  // U = W_c / sigma (mr = n1 rows) and V = V_c (nc = n2 rows); with it the roles swap.
  const int k = d.k;
  T* U = uhat + int64_t(slice) * d.n1 * k;
  T* Vo = vhat + int64_t(slice) * d.n2 * k;
  T* Us = us + int64_t(slice) * d.n1 * k;
  for (int i = wave; i < k; i += kJacobiWaves) {
    const int c = s_order[i];
    const double sg = s_sigma[c];
    const double inv = sg > 0 ? 1.0 / sg : 0.0;
    // Values of the final U column: either W_c * inv or V_c.
    auto ucol = [&](int row) -> double {
      return d.trans ? double(V[int64_t(c) * nc + row]) : double(W[int64_t(c) * mr + row]) * inv;
    };
    auto vcol = [&](int row) -> double {
      return d.trans ? double(W[int64_t(c) * mr + row]) * inv : double(V[int64_t(c) * nc + row]);
    };
    // Largest |U| entry, lowest row on ties.
    double best = -1.0;
    int brow = 0x7fffffff;
    double bval = 0;
    for (int row = lane; row < d.n1; row += 64) {
      const double x = ucol(row);
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
    for (int row = lane; row < d.n1; row += 64) {
      const double x = sgn * ucol(row);
      U[int64_t(row) * k + i] = T(x);
      Us[int64_t(row) * k + i] = T(T(x) * T(sg));
    }
    for (int row = lane; row < d.n2; row += 64) Vo[int64_t(row) * k + i] = T(sgn * vcol(row));
    if (lane == 0) shat[int64_t(slice) * k + i] = T(sg);
  }
  if (threadIdx.x == 0) info[slice] = (converged && s_bad == 0) ? sweeps : -sweeps;
}

// max |X^T X - I| over the k x k Gram matrix of one slice of X (n x k, row-major), FP64.
template <typename T>
__global__ __launch_bounds__(256) void orth_kernel(const T* __restrict__ x, int n, int k,
                                                   double* __restrict__ part) {
  const int slice = blockIdx.x;
  const T* X = x + int64_t(slice) * n * k;
  double worst = 0;
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int a = e / k, b = e % k;
    if (b < a) continue;
    double acc = 0;
    for (int r = 0; r < n; ++r) acc = fma(double(X[int64_t(r) * k + a]), double(X[int64_t(r) * k + b]), acc);
    const double dev = fabs(acc - (a == b ? 1.0 : 0.0));
    worst = (dev > worst || dev != dev) ? dev : worst;
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
  if (threadIdx.x == 0) part[slice] = red[0];
}

__global__ __launch_bounds__(256) void max_reduce_kernel(const double* __restrict__ part, int64_t n,
                                                         double* __restrict__ out) {
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
  if (threadIdx.x == 0) *out = red[0];
}

struct SvdPlan {
  size_t ah, w, v, us, part, total;
};

inline SvdPlan plan_svd(int64_t n1, int64_t n2, int64_t p, int k, size_t es) {
  const int64_t mr = n1 > n2 ? n1 : n2;
  const int64_t nc = n1 > n2 ? n2 : n1;
  SvdPlan pl{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  pl.ah = take(size_t(p * n1 * n2) * es);  // coefficients, later the rebuilt ones
  pl.w = take(size_t(p * nc * mr) * es);
  pl.v = take(size_t(p * nc * nc) * es);
  pl.us = take(size_t(p * n1 * k) * es);
  pl.part = take(size_t(p) * 2 * sizeof(double));
  pl.total = off + 256;
  return pl;
}

template <typename T>
hipError_t run_svd(const T* a, int64_t n1, int64_t n2, int64_t p, int L, int k, T* uhat, T* shat,
                   T* vhat, T* ak, int max_sweeps, int32_t* info, double* orth_err, void* ws,
                   hipStream_t s) {
  const SvdPlan pl = plan_svd(n1, n2, p, k, sizeof(T));
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
  T* ah = reinterpret_cast<T*>(base + pl.ah);
  T* w = reinterpret_cast<T*>(base + pl.w);
  T* v = reinterpret_cast<T*>(base + pl.v);
  T* us = reinterpret_cast<T*>(base + pl.us);
  double* part = reinterpret_cast<double*>(base + pl.part);

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

  const dim3 grid{unsigned(p)};
  const dim3 block{unsigned(kJacobiThreads)};
  if (d.mr <= 64)
    hipLaunchKernelGGL((jacobi_kernel<T, 1>), grid, block, 0, s, ah, w, v, d, max_sweeps, uhat, shat, vhat, us, info);
  else if (d.mr <= 128)
    hipLaunchKernelGGL((jacobi_kernel<T, 2>), grid, block, 0, s, ah, w, v, d, max_sweeps, uhat, shat, vhat, us, info);
  else if (d.mr <= 256)
    hipLaunchKernelGGL((jacobi_kernel<T, 4>), grid, block, 0, s, ah, w, v, d, max_sweeps, uhat, shat, vhat, us, info);
  else if (d.mr <= 512)
    hipLaunchKernelGGL((jacobi_kernel<T, 8>), grid, block, 0, s, ah, w, v, d, max_sweeps, uhat, shat, vhat, us, info);
  else
    hipLaunchKernelGGL((jacobi_kernel<T, 16>), grid, block, 0, s, ah, w, v, d, max_sweeps, uhat, shat, vhat, us, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  if (ak != nullptr) {
    // Rebuild Chat = (U sigma) V^T per slice (a face-product with inner size k),
    // reusing the coefficient region, then W^{-1}.
    if constexpr (sizeof(T) == 8) {
      e = launch_face_f64(reinterpret_cast<const double*>(us), reinterpret_cast<const double*>(vhat),
                          reinterpret_cast<double*>(ah), n1, k, n2, p, false, true, s);
      if (e == hipSuccess)
        e = launch_lift_f64(LiftKind::kInverse, reinterpret_cast<const double*>(ah),
                            reinterpret_cast<double*>(ak), n1 * n2, p, L, s);
    } else {
      e = launch_face_f32(reinterpret_cast<const float*>(us), reinterpret_cast<const float*>(vhat),
                          reinterpret_cast<float*>(ah), n1, k, n2, p, false, true, s);
      if (e == hipSuccess)
        e = launch_lift_f32(LiftKind::kInverse, reinterpret_cast<const float*>(ah),
                            reinterpret_cast<float*>(ak), n1 * n2, p, L, s);
    }
    if (e != hipSuccess) return e;
  }

  if (orth_err != nullptr) {
    hipLaunchKernelGGL((orth_kernel<T>), dim3(unsigned(p)), dim3(256), 0, s, uhat, int(n1), k, part);
    hipLaunchKernelGGL((orth_kernel<T>), dim3(unsigned(p)), dim3(256), 0, s, vhat, int(n2), k, part + p);
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, part, p, orth_err);
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, part + p, p, orth_err + 1);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

size_t svd_workspace_bytes(int64_t n1, int64_t n2, int64_t p, int k, int dtype) {
  return plan_svd(n1, n2, p, k, dtype == 0 ? 8 : 4).total;
}

hipError_t launch_svd(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k, void* uhat,
                      void* shat, void* vhat, void* ak, int max_sweeps, int32_t* info,
                      double* orth_err, int dtype, void* ws, hipStream_t s) {
  if (dtype == 0)
    return run_svd<double>(static_cast<const double*>(a), n1, n2, p, L, k, static_cast<double*>(uhat),
                           static_cast<double*>(shat), static_cast<double*>(vhat),
                           static_cast<double*>(ak), max_sweeps, info, orth_err, ws, s);
  return run_svd<float>(static_cast<const float*>(a), n1, n2, p, L, k, static_cast<float*>(uhat),
                        static_cast<float*>(shat), static_cast<float*>(vhat), static_cast<float*>(ak),
                        max_sweeps, info, orth_err, ws, s);
}

}  // namespace wp
