// Internal declarations shared by the HIP sources of libwprod.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wp {

// Which lifting-type pass to run over the mode-3 tubes.
enum class LiftKind : int {
  kForward = 0,     // W      : spatial -> coefficients
  kInverse = 1,     // W^{-1} : coefficients -> spatial
  kForwardAdj = 2,  // W^T    : coefficients -> spatial
  kInverseAdj = 3,  // W^{-T} : spatial -> coefficients
};

// Output format of a pass that produces coefficients from float data.
enum class StoreKind : int {
  kPlain = 0,  // same dtype as the input
  kSplit = 1,  // bf16 hi (+ optional lo) bit patterns
};

// Largest supported level count (two register tiers of five levels).
constexpr int kMaxLevels = 10;

// Lifting passes.  All pointers device, tensors (p, n1*n2) with P = n1*n2.
hipError_t launch_lift_f64(LiftKind kind, const double* in, double* out, int64_t P, int64_t p,
                           int L, hipStream_t s);
hipError_t launch_lift_f32(LiftKind kind, const float* in, float* out, int64_t P, int64_t p,
                           int L, hipStream_t s);
hipError_t launch_lift_f32_split(LiftKind kind, const float* in, uint16_t* hi, uint16_t* lo,
                                 int64_t P, int64_t p, int L, hipStream_t s);

// Lifting with chosen predict / update stencils (scheme.hip).  taps.w[j-1][0]
// is the predict and taps.w[j-1][1] the update stencil of level j, tap t at
// offset t - 2.
struct SchemeTaps {
  double w[kMaxLevels][2][5];
};
// Positions per workgroup tile for p slices of es bytes (0: p too large).
int scheme_tile_positions(int64_t p, size_t es);
hipError_t launch_lift_scheme_f64(LiftKind kind, const double* in, double* out, int64_t P,
                                  int64_t p, int L, const SchemeTaps& taps, hipStream_t s);
hipError_t launch_lift_scheme_f32(LiftKind kind, const float* in, float* out, int64_t P,
                                  int64_t p, int L, const SchemeTaps& taps, hipStream_t s);
// Forward or W^{-T} pass of float data written as bf16 hi (+ optional lo) planes.
hipError_t launch_lift_scheme_f32_split(LiftKind kind, const float* in, uint16_t* hi,
                                        uint16_t* lo, int64_t P, int64_t p, int L,
                                        const SchemeTaps& taps, hipStream_t s);

// Face-product GEMMs.  C[k] = op(A[k]) op(B[k]), op(A) m x kk, op(B) kk x n.
hipError_t launch_face_f64(const double* a, const double* b, double* c, int64_t m, int64_t kk,
                           int64_t n, int64_t batch, bool ta, bool tb, hipStream_t s);
hipError_t launch_face_f32(const float* a, const float* b, float* c, int64_t m, int64_t kk,
                           int64_t n, int64_t batch, bool ta, bool tb, hipStream_t s);
hipError_t launch_face_bf16(const uint16_t* ahi, const uint16_t* alo, const uint16_t* bhi,
                            const uint16_t* blo, float* c, int64_t m, int64_t kk, int64_t n,
                            int64_t batch, bool ta, bool tb, bool x3, hipStream_t s);

// w-svd pieces (see svd.hip).
// sparse = true decomposes only s_L and d_L (sp-w-svd); outputs then hold
// 2 p / 2^L slices.
size_t svd_workspace_bytes(int64_t n1, int64_t n2, int64_t p, int L, int k, bool sparse,
                           int dtype);
// ev_begin / ev_end (may be null) are recorded on s just before and just after
// the Jacobi stage.
hipError_t launch_svd(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                      bool sparse, void* uhat, void* shat, void* vhat, void* ak, int max_sweeps,
                      int32_t* info, double* orth_err, int dtype, void* ws, hipStream_t s,
                      hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);

// Moore-Penrose inverse (Def. 2.6) through the same SVD; out is (p, n2, n1).
size_t pinv_workspace_bytes(int64_t n1, int64_t n2, int64_t p, int L, bool sparse, int dtype);
hipError_t launch_pinv(const void* a, void* out, int64_t n1, int64_t n2, int64_t p, int L,
                       bool sparse, double rtol, int32_t* info, int dtype, void* ws, hipStream_t s);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace wp
