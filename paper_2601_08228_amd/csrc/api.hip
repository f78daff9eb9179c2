// extern "C" entry points of libwprod.so: argument validation (before any HIP
// call), workspace carving and kernel dispatch.  See include/wprod.h for the
// contract of each call.

#include <mutex>

#include "wprod.h"
#include "wp_internal.h"

// Device scratch of w_product_noalloc: one fixed array, 256-byte aligned, on
// every device the library runs on, held until the process ends.  Host code
// never passes the name `scratch` to a kernel or a copy (on the host it only
// names the symbol); it uses the device address that hipGetSymbolAddress
// returns for the current device (scratch_on_current_device below).
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

using wp::LiftKind;

constexpr int64_t kMaxElems = int64_t(1) << 40;
constexpr size_t kAlign = 256;

struct Range {
  const char* lo;
  const char* hi;
};

inline Range range_of(const void* p, int64_t elems, size_t esize) {
  const char* c = static_cast<const char*>(p);
  return Range{c, c + size_t(elems) * esize};
}

inline bool overlap(const Range& a, const Range& b) {
  return a.lo != nullptr && b.lo != nullptr && a.lo < b.hi && b.lo < a.hi;
}

inline size_t dtype_size(int dtype) { return dtype == WP_F64 ? 8 : 4; }

inline bool valid_dtype(int dtype) { return dtype == WP_F64 || dtype == WP_F32; }

// Product of positive sizes with an overflow guard; -1 if too large.
inline int64_t checked_mul(int64_t a, int64_t b) {
  if (a <= 0 || b <= 0) return -1;
  if (a > kMaxElems / b) return -1;
  return a * b;
}

inline wp_status check_tensor(int64_t n1, int64_t n2, int64_t p, int L, int64_t* elems) {
  if (n1 < 1 || n2 < 1 || p < 1) return WP_EINVAL;
  if (L < 0 || L > wp::kMaxLevels) return WP_EINVAL;
  if (p % (int64_t(1) << L) != 0) return WP_EINVAL;
  const int64_t e = checked_mul(checked_mul(n1, n2), p);
  if (e < 0) return WP_EINVAL;
  if (n1 > INT32_MAX || n2 > INT32_MAX) return WP_EINVAL;
  *elems = e;
  return WP_OK;
}

inline wp_status from_hip(hipError_t e) { return e == hipSuccess ? WP_OK : WP_ELAUNCH; }

wp_status run_lift(LiftKind kind, const void* in, void* out, int64_t n1, int64_t n2, int64_t p,
                   int L, int dtype, void* stream) {
  if (!valid_dtype(dtype)) return WP_EDTYPE;
  int64_t elems = 0;
  wp_status st = check_tensor(n1, n2, p, L, &elems);
  if (st != WP_OK) return st;
  if (in == nullptr || out == nullptr) return WP_ENULL;
  const size_t es = dtype_size(dtype);
  if (overlap(range_of(in, elems, es), range_of(out, elems, es))) return WP_EALIAS;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == WP_F64)
    return from_hip(wp::launch_lift_f64(kind, static_cast<const double*>(in),
                                        static_cast<double*>(out), n1 * n2, p, L, s));
  return from_hip(wp::launch_lift_f32(kind, static_cast<const float*>(in), static_cast<float*>(out),
                                      n1 * n2, p, L, s));
}

wp_status run_lift_split(LiftKind kind, const float* in, uint16_t* hi, uint16_t* lo, int64_t n1,
                         int64_t n2, int64_t p, int L, void* stream) {
  int64_t elems = 0;
  wp_status st = check_tensor(n1, n2, p, L, &elems);
  if (st != WP_OK) return st;
  if (in == nullptr || hi == nullptr) return WP_ENULL;
  const Range rin = range_of(in, elems, 4);
  const Range rhi = range_of(hi, elems, 2);
  const Range rlo = range_of(lo, elems, 2);
  if (overlap(rin, rhi) || overlap(rin, rlo) || overlap(rhi, rlo)) return WP_EALIAS;
  return from_hip(wp::launch_lift_f32_split(kind, in, hi, lo, n1 * n2, p, L,
                                            static_cast<hipStream_t>(stream)));
}

// Sizes of the three face-product operands, in elements.
struct FaceShapes {
  int64_t a, b, c;
};

inline wp_status check_face(int64_t n1, int64_t n2, int64_t n3, int64_t p, int ta, int tb,
                            FaceShapes* fs) {
  if (n1 < 1 || n2 < 1 || n3 < 1 || p < 1) return WP_EINVAL;
  if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) return WP_EINVAL;
  if (n1 > INT32_MAX || n2 > INT32_MAX || n3 > INT32_MAX) return WP_EINVAL;
  fs->a = checked_mul(checked_mul(n1, n2), p);
  fs->b = checked_mul(checked_mul(n2, n3), p);
  fs->c = checked_mul(checked_mul(n1, n3), p);
  if (fs->a < 0 || fs->b < 0 || fs->c < 0) return WP_EINVAL;
  return WP_OK;
}

struct ProductPlan {
  size_t ah, ah_lo, bh, bh_lo, ch, total;  // byte offsets into the aligned workspace
};

// Workspace layout of w_product: transformed A, transformed B (split planes
// for the BF16 modes), transformed C; each region 256-byte aligned, plus
// 256 bytes of slack so that any caller alignment works.
inline ProductPlan plan_product(const FaceShapes& fs, int dtype, int gemm) {
  ProductPlan pl{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = wp::align_up(off + bytes, kAlign);
    return at;
  };
  if (gemm == WP_GEMM_NATIVE) {
    const size_t es = dtype_size(dtype);
    pl.ah = take(size_t(fs.a) * es);
    pl.bh = take(size_t(fs.b) * es);
    pl.ch = take(size_t(fs.c) * es);
  } else {
    pl.ah = take(size_t(fs.a) * 2);
    pl.ah_lo = gemm == WP_GEMM_BF16X3 ? take(size_t(fs.a) * 2) : 0;
    pl.bh = take(size_t(fs.b) * 2);
    pl.bh_lo = gemm == WP_GEMM_BF16X3 ? take(size_t(fs.b) * 2) : 0;
    pl.ch = take(size_t(fs.c) * 4);
  }
  pl.total = off + kAlign;
  return pl;
}

// Workspace layout of w_face_product_gemm: the bf16 planes of both operands
// (no transformed C; native mode needs no workspace).
inline ProductPlan plan_face(const FaceShapes& fs, int gemm) {
  ProductPlan pl{};
  if (gemm == WP_GEMM_NATIVE) return pl;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = wp::align_up(off + bytes, kAlign);
    return at;
  };
  pl.ah = take(size_t(fs.a) * 2);
  pl.ah_lo = gemm == WP_GEMM_BF16X3 ? take(size_t(fs.a) * 2) : 0;
  pl.bh = take(size_t(fs.b) * 2);
  pl.bh_lo = gemm == WP_GEMM_BF16X3 ? take(size_t(fs.b) * 2) : 0;
  pl.total = off + kAlign;
  return pl;
}

// Host taps (L levels x {predict, update} x 5) into the kernel argument; every
// tap finite.  L = 0 needs no taps.
inline wp_status load_taps(const double* taps, int L, wp::SchemeTaps* out) {
  *out = wp::SchemeTaps{};
  if (L == 0) return WP_OK;
  if (taps == nullptr) return WP_ENULL;
  for (int j = 0; j < L; ++j)
    for (int k = 0; k < 2; ++k)
      for (int t = 0; t < WP_TAPS; ++t) {
        const double v = taps[(j * 2 + k) * WP_TAPS + t];
        if (!(v - v == 0.0)) return WP_EINVAL;  // NaN or infinite
        out->w[j][k][t] = v;
      }
  return WP_OK;
}

inline bool scheme_fits(int64_t p, int dtype) {
  return wp::scheme_tile_positions(p, dtype_size(dtype)) != 0;
}

inline LiftKind lift_kind(int kind) {
  switch (kind) {
    case WP_LIFT_INVERSE: return LiftKind::kInverse;
    case WP_LIFT_ADJ: return LiftKind::kForwardAdj;
    case WP_LIFT_IADJ: return LiftKind::kInverseAdj;
    default: return LiftKind::kForward;
  }
}

inline wp_status check_modes(int dtype, int gemm) {
  if (!valid_dtype(dtype)) return WP_EDTYPE;
  if (gemm != WP_GEMM_NATIVE && gemm != WP_GEMM_BF16 && gemm != WP_GEMM_BF16X3) return WP_EDTYPE;
  if (gemm != WP_GEMM_NATIVE && dtype != WP_F32) return WP_EDTYPE;
  return WP_OK;
}

// Device address of `scratch` on the calling thread's current device, looked
// up once per device (with that device current) and kept.
constexpr int kMaxDevices = 64;
struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxDevices];

wp_status scratch_on_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return WP_ELAUNCH;
  ScratchSlot& sl = g_scratch[dev];
  std::call_once(sl.once, [&sl] {
    sl.err = hipGetSymbolAddress(&sl.ptr, HIP_SYMBOL(scratch));
  });
  if (sl.err != hipSuccess || sl.ptr == nullptr) return WP_ELAUNCH;
  *out = sl.ptr;
  return WP_OK;
}

// Enqueues the w-product on `stream` with the workspace `ws` laid out by pl
// (arguments already validated).
wp_status enqueue_product(const void* a, const void* b, void* c, int64_t n1, int64_t n2,
                          int64_t n3, int64_t p, int L, int trans_a, int trans_b, int dtype,
                          int gemm, const ProductPlan& pl, void* ws, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(wp::align_up(reinterpret_cast<uintptr_t>(ws), kAlign));
  // Stored shapes: A is (p, n1, n2) or (p, n2, n1); the transform only sees
  // n1*n2 positions per slice either way (Thm 2.1).
  const int64_t Pa = n1 * n2, Pb = n2 * n3, Pc = n1 * n3;
  hipError_t e = hipSuccess;
  if (gemm == WP_GEMM_NATIVE) {
    void* ah = base + pl.ah;
    void* bh = base + pl.bh;
    void* ch = base + pl.ch;
    if (dtype == WP_F64) {
      e = wp::launch_lift_f64(LiftKind::kForward, static_cast<const double*>(a), static_cast<double*>(ah), Pa, p, L, s);
      if (e == hipSuccess) e = wp::launch_lift_f64(LiftKind::kForward, static_cast<const double*>(b), static_cast<double*>(bh), Pb, p, L, s);
      if (e == hipSuccess) e = wp::launch_face_f64(static_cast<const double*>(ah), static_cast<const double*>(bh), static_cast<double*>(ch), n1, n2, n3, p, trans_a != 0, trans_b != 0, s);
      if (e == hipSuccess) e = wp::launch_lift_f64(LiftKind::kInverse, static_cast<const double*>(ch), static_cast<double*>(c), Pc, p, L, s);
    } else {
      e = wp::launch_lift_f32(LiftKind::kForward, static_cast<const float*>(a), static_cast<float*>(ah), Pa, p, L, s);
      if (e == hipSuccess) e = wp::launch_lift_f32(LiftKind::kForward, static_cast<const float*>(b), static_cast<float*>(bh), Pb, p, L, s);
      if (e == hipSuccess) e = wp::launch_face_f32(static_cast<const float*>(ah), static_cast<const float*>(bh), static_cast<float*>(ch), n1, n2, n3, p, trans_a != 0, trans_b != 0, s);
      if (e == hipSuccess) e = wp::launch_lift_f32(LiftKind::kInverse, static_cast<const float*>(ch), static_cast<float*>(c), Pc, p, L, s);
    }
  } else {
    const bool x3 = gemm == WP_GEMM_BF16X3;
    uint16_t* ahi = reinterpret_cast<uint16_t*>(base + pl.ah);
    uint16_t* alo = x3 ? reinterpret_cast<uint16_t*>(base + pl.ah_lo) : nullptr;
    uint16_t* bhi = reinterpret_cast<uint16_t*>(base + pl.bh);
    uint16_t* blo = x3 ? reinterpret_cast<uint16_t*>(base + pl.bh_lo) : nullptr;
    float* ch = reinterpret_cast<float*>(base + pl.ch);
    e = wp::launch_lift_f32_split(LiftKind::kForward, static_cast<const float*>(a), ahi, alo, Pa, p, L, s);
    if (e == hipSuccess) e = wp::launch_lift_f32_split(LiftKind::kForward, static_cast<const float*>(b), bhi, blo, Pb, p, L, s);
    if (e == hipSuccess) e = wp::launch_face_bf16(ahi, alo, bhi, blo, ch, n1, n2, n3, p, trans_a != 0, trans_b != 0, x3, s);
    if (e == hipSuccess) e = wp::launch_lift_f32(LiftKind::kInverse, ch, static_cast<float*>(c), Pc, p, L, s);
  }
  return from_hip(e);
}


}  // namespace

extern "C" {

const char* w_status_string(wp_status s) {
  switch (s) {
    case WP_OK: return "WP_OK";
    case WP_EINVAL: return "WP_EINVAL: invalid size, level, rank or flag";
    case WP_ENULL: return "WP_ENULL: required pointer is NULL";
    case WP_EALIAS: return "WP_EALIAS: an output overlaps an input or another output";
    case WP_EDTYPE: return "WP_EDTYPE: unknown dtype or GEMM mode not valid for the dtype";
    case WP_EWORKSPACE: return "WP_EWORKSPACE: workspace too small";
    case WP_ELAUNCH: return "WP_ELAUNCH: HIP launch or runtime call failed";
    case WP_ENOCONV: return "WP_ENOCONV: a Jacobi slice did not converge";
    case WP_ESCRATCH:
      return "WP_ESCRATCH: the call needs more device scratch than w_product_noalloc holds";
  }
  return "unknown wp_status";
}

int w_version(void) { return 100; }

wp_status w_transform(const void* x, void* xhat, int64_t n1, int64_t n2, int64_t p, int L,
                      int dtype, void* stream) {
  return run_lift(LiftKind::kForward, x, xhat, n1, n2, p, L, dtype, stream);
}

wp_status w_itransform(const void* xhat, void* x, int64_t n1, int64_t n2, int64_t p, int L,
                       int dtype, void* stream) {
  return run_lift(LiftKind::kInverse, xhat, x, n1, n2, p, L, dtype, stream);
}

wp_status w_transform_adj(const void* g, void* out, int64_t n1, int64_t n2, int64_t p, int L,
                          int dtype, void* stream) {
  return run_lift(LiftKind::kForwardAdj, g, out, n1, n2, p, L, dtype, stream);
}

wp_status w_itransform_adj(const void* g, void* out, int64_t n1, int64_t n2, int64_t p, int L,
                           int dtype, void* stream) {
  return run_lift(LiftKind::kInverseAdj, g, out, n1, n2, p, L, dtype, stream);
}

wp_status w_transform_split(const float* x, uint16_t* xhat_hi, uint16_t* xhat_lo, int64_t n1,
                            int64_t n2, int64_t p, int L, void* stream) {
  return run_lift_split(LiftKind::kForward, x, xhat_hi, xhat_lo, n1, n2, p, L, stream);
}

wp_status w_itransform_adj_split(const float* g, uint16_t* out_hi, uint16_t* out_lo, int64_t n1,
                                 int64_t n2, int64_t p, int L, void* stream) {
  return run_lift_split(LiftKind::kInverseAdj, g, out_hi, out_lo, n1, n2, p, L, stream);
}

wp_status w_face_product(const void* ah, const void* bh, void* ch, int64_t n1, int64_t n2,
                         int64_t n3, int64_t p, int trans_a, int trans_b, int dtype,
                         void* stream) {
  if (!valid_dtype(dtype)) return WP_EDTYPE;
  FaceShapes fs{};
  wp_status st = check_face(n1, n2, n3, p, trans_a, trans_b, &fs);
  if (st != WP_OK) return st;
  if (ah == nullptr || bh == nullptr || ch == nullptr) return WP_ENULL;
  const size_t es = dtype_size(dtype);
  const Range rc = range_of(ch, fs.c, es);
  if (overlap(rc, range_of(ah, fs.a, es)) || overlap(rc, range_of(bh, fs.b, es))) return WP_EALIAS;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == WP_F64)
    return from_hip(wp::launch_face_f64(static_cast<const double*>(ah), static_cast<const double*>(bh),
                                        static_cast<double*>(ch), n1, n2, n3, p, trans_a != 0,
                                        trans_b != 0, s));
  return from_hip(wp::launch_face_f32(static_cast<const float*>(ah), static_cast<const float*>(bh),
                                      static_cast<float*>(ch), n1, n2, n3, p, trans_a != 0,
                                      trans_b != 0, s));
}

wp_status w_face_product_split(const uint16_t* a_hi, const uint16_t* a_lo, const uint16_t* b_hi,
                               const uint16_t* b_lo, float* ch, int64_t n1, int64_t n2, int64_t n3,
                               int64_t p, int trans_a, int trans_b, int gemm, void* stream) {
  if (gemm != WP_GEMM_BF16 && gemm != WP_GEMM_BF16X3) return WP_EDTYPE;
  FaceShapes fs{};
  wp_status st = check_face(n1, n2, n3, p, trans_a, trans_b, &fs);
  if (st != WP_OK) return st;
  const bool x3 = gemm == WP_GEMM_BF16X3;
  if (a_hi == nullptr || b_hi == nullptr || ch == nullptr) return WP_ENULL;
  if (x3 && (a_lo == nullptr || b_lo == nullptr)) return WP_ENULL;
  const Range rc = range_of(ch, fs.c, 4);
  if (overlap(rc, range_of(a_hi, fs.a, 2)) || overlap(rc, range_of(b_hi, fs.b, 2))) return WP_EALIAS;
  if (x3 && (overlap(rc, range_of(a_lo, fs.a, 2)) || overlap(rc, range_of(b_lo, fs.b, 2))))
    return WP_EALIAS;
  return from_hip(wp::launch_face_bf16(a_hi, a_lo, b_hi, b_lo, ch, n1, n2, n3, p, trans_a != 0,
                                       trans_b != 0, x3, static_cast<hipStream_t>(stream)));
}

size_t w_face_product_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int dtype,
                                int gemm) {
  if (check_modes(dtype, gemm) != WP_OK) return 0;
  FaceShapes fs{};
  if (check_face(n1, n2, n3, p, 0, 0, &fs) != WP_OK) return 0;
  return plan_face(fs, gemm).total;
}

wp_status w_face_product_gemm(const void* ah, const void* bh, void* ch, int64_t n1, int64_t n2,
                              int64_t n3, int64_t p, int trans_a, int trans_b, int dtype,
                              int gemm, void* ws, size_t ws_bytes, void* stream) {
  wp_status st = check_modes(dtype, gemm);
  if (st != WP_OK) return st;
  if (gemm == WP_GEMM_NATIVE)
    return w_face_product(ah, bh, ch, n1, n2, n3, p, trans_a, trans_b, dtype, stream);
  FaceShapes fs{};
  st = check_face(n1, n2, n3, p, trans_a, trans_b, &fs);
  if (st != WP_OK) return st;
  if (ah == nullptr || bh == nullptr || ch == nullptr || ws == nullptr) return WP_ENULL;
  const ProductPlan pl = plan_face(fs, gemm);
  if (ws_bytes < pl.total) return WP_EWORKSPACE;
  const Range ra = range_of(ah, fs.a, 4), rb = range_of(bh, fs.b, 4), rc = range_of(ch, fs.c, 4);
  const Range rw{static_cast<const char*>(ws), static_cast<const char*>(ws) + ws_bytes};
  if (overlap(rc, ra) || overlap(rc, rb) || overlap(rw, ra) || overlap(rw, rb) || overlap(rw, rc))
    return WP_EALIAS;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(wp::align_up(reinterpret_cast<uintptr_t>(ws), kAlign));
  const bool x3 = gemm == WP_GEMM_BF16X3;
  uint16_t* ahi = reinterpret_cast<uint16_t*>(base + pl.ah);
  uint16_t* alo = x3 ? reinterpret_cast<uint16_t*>(base + pl.ah_lo) : nullptr;
  uint16_t* bhi = reinterpret_cast<uint16_t*>(base + pl.bh);
  uint16_t* blo = x3 ? reinterpret_cast<uint16_t*>(base + pl.bh_lo) : nullptr;
  // The split is elementwise: the identity transform (L = 0) with the
  // split epilogue, over whatever stored shape the operands have.
  hipError_t e = wp::launch_lift_f32_split(LiftKind::kForward, static_cast<const float*>(ah), ahi,
                                           alo, n1 * n2, p, 0, s);
  if (e == hipSuccess)
    e = wp::launch_lift_f32_split(LiftKind::kForward, static_cast<const float*>(bh), bhi, blo,
                                  n2 * n3, p, 0, s);
  if (e == hipSuccess)
    e = wp::launch_face_bf16(ahi, alo, bhi, blo, static_cast<float*>(ch), n1, n2, n3, p,
                             trans_a != 0, trans_b != 0, x3, s);
  return from_hip(e);
}

size_t w_product_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int L, int dtype,
                           int gemm) {
  if (check_modes(dtype, gemm) != WP_OK) return 0;
  FaceShapes fs{};
  if (check_face(n1, n2, n3, p, 0, 0, &fs) != WP_OK) return 0;
  if (L < 0 || L > wp::kMaxLevels || p % (int64_t(1) << L) != 0) return 0;
  return plan_product(fs, dtype, gemm).total;
}

wp_status w_product(const void* a, const void* b, void* c, int64_t n1, int64_t n2, int64_t n3,
                    int64_t p, int L, int trans_a, int trans_b, int dtype, int gemm, void* ws,
                    size_t ws_bytes, void* stream) {
  wp_status st = check_modes(dtype, gemm);
  if (st != WP_OK) return st;
  FaceShapes fs{};
  st = check_face(n1, n2, n3, p, trans_a, trans_b, &fs);
  if (st != WP_OK) return st;
  if (L < 0 || L > wp::kMaxLevels || p % (int64_t(1) << L) != 0) return WP_EINVAL;
  if (a == nullptr || b == nullptr || c == nullptr || ws == nullptr) return WP_ENULL;
  const ProductPlan pl = plan_product(fs, dtype, gemm);
  if (ws_bytes < pl.total) return WP_EWORKSPACE;
  const size_t es = dtype_size(dtype);
  const Range ra = range_of(a, fs.a, es), rb = range_of(b, fs.b, es), rc = range_of(c, fs.c, es);
  const Range rw{static_cast<const char*>(ws), static_cast<const char*>(ws) + ws_bytes};
  if (overlap(rc, ra) || overlap(rc, rb) || overlap(rw, ra) || overlap(rw, rb) || overlap(rw, rc))
    return WP_EALIAS;

  return enqueue_product(a, b, c, n1, n2, n3, p, L, trans_a, trans_b, dtype, gemm, pl, ws, stream);
}

size_t w_product_noalloc_scratch_bytes(void) { return kScratchBytes; }

wp_status w_product_noalloc(const void* a, const void* b, void* c, int64_t n1, int64_t n2,
                            int64_t n3, int64_t p, int L, int trans_a, int trans_b, int dtype,
                            int gemm, void* stream) {
  wp_status st = check_modes(dtype, gemm);
  if (st != WP_OK) return st;
  FaceShapes fs{};
  st = check_face(n1, n2, n3, p, trans_a, trans_b, &fs);
  if (st != WP_OK) return st;
  if (L < 0 || L > wp::kMaxLevels || p % (int64_t(1) << L) != 0) return WP_EINVAL;
  const ProductPlan pl = plan_product(fs, dtype, gemm);
  if (pl.total > kScratchBytes) return WP_ESCRATCH;
  if (a == nullptr || b == nullptr || c == nullptr) return WP_ENULL;
  const size_t es = dtype_size(dtype);
  const Range ra = range_of(a, fs.a, es), rb = range_of(b, fs.b, es), rc = range_of(c, fs.c, es);
  if (overlap(rc, ra) || overlap(rc, rb)) return WP_EALIAS;
  void* ws = nullptr;
  st = scratch_on_current_device(&ws);
  if (st != WP_OK) return st;
  return enqueue_product(a, b, c, n1, n2, n3, p, L, trans_a, trans_b, dtype, gemm, pl, ws, stream);
}

wp_status w_transform_scheme(const void* in, void* out, int64_t n1, int64_t n2, int64_t p, int L,
                             const double* taps, int kind, int dtype, void* stream) {
  if (!valid_dtype(dtype)) return WP_EDTYPE;
  int64_t elems = 0;
  wp_status st = check_tensor(n1, n2, p, L, &elems);
  if (st != WP_OK) return st;
  if (kind < WP_LIFT_FORWARD || kind > WP_LIFT_IADJ || !scheme_fits(p, dtype)) return WP_EINVAL;
  wp::SchemeTaps tp{};
  st = load_taps(taps, L, &tp);
  if (st != WP_OK) return st;
  if (in == nullptr || out == nullptr) return WP_ENULL;
  const size_t es = dtype_size(dtype);
  if (overlap(range_of(in, elems, es), range_of(out, elems, es))) return WP_EALIAS;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == WP_F64)
    return from_hip(wp::launch_lift_scheme_f64(lift_kind(kind), static_cast<const double*>(in),
                                               static_cast<double*>(out), n1 * n2, p, L, tp, s));
  return from_hip(wp::launch_lift_scheme_f32(lift_kind(kind), static_cast<const float*>(in),
                                             static_cast<float*>(out), n1 * n2, p, L, tp, s));
}

wp_status w_transform_scheme_split(const float* in, uint16_t* out_hi, uint16_t* out_lo,
                                   int64_t n1, int64_t n2, int64_t p, int L, const double* taps,
                                   int kind, void* stream) {
  int64_t elems = 0;
  wp_status st = check_tensor(n1, n2, p, L, &elems);
  if (st != WP_OK) return st;
  if ((kind != WP_LIFT_FORWARD && kind != WP_LIFT_IADJ) || !scheme_fits(p, WP_F32))
    return WP_EINVAL;
  wp::SchemeTaps tp{};
  st = load_taps(taps, L, &tp);
  if (st != WP_OK) return st;
  if (in == nullptr || out_hi == nullptr) return WP_ENULL;
  const Range rin = range_of(in, elems, 4);
  const Range rhi = range_of(out_hi, elems, 2);
  const Range rlo = range_of(out_lo, elems, 2);
  if (overlap(rin, rhi) || overlap(rin, rlo) || overlap(rhi, rlo)) return WP_EALIAS;
  return from_hip(wp::launch_lift_scheme_f32_split(lift_kind(kind), in, out_hi, out_lo, n1 * n2,
                                                   p, L, tp, static_cast<hipStream_t>(stream)));
}

size_t w_product_scheme_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int L,
                                  int dtype, int gemm) {
  if (!valid_dtype(dtype) || !scheme_fits(p, dtype)) return 0;
  return w_product_workspace(n1, n2, n3, p, L, dtype, gemm);
}

wp_status w_product_scheme(const void* a, const void* b, void* c, int64_t n1, int64_t n2,
                           int64_t n3, int64_t p, int L, const double* taps, int trans_a,
                           int trans_b, int dtype, int gemm, void* ws, size_t ws_bytes,
                           void* stream) {
  wp_status st = check_modes(dtype, gemm);
  if (st != WP_OK) return st;
  FaceShapes fs{};
  st = check_face(n1, n2, n3, p, trans_a, trans_b, &fs);
  if (st != WP_OK) return st;
  if (L < 0 || L > wp::kMaxLevels || p % (int64_t(1) << L) != 0) return WP_EINVAL;
  if (!scheme_fits(p, dtype)) return WP_EINVAL;
  wp::SchemeTaps tp{};
  st = load_taps(taps, L, &tp);
  if (st != WP_OK) return st;
  if (a == nullptr || b == nullptr || c == nullptr || ws == nullptr) return WP_ENULL;
  const ProductPlan pl = plan_product(fs, dtype, gemm);
  if (ws_bytes < pl.total) return WP_EWORKSPACE;
  const size_t es = dtype_size(dtype);
  const Range ra = range_of(a, fs.a, es), rb = range_of(b, fs.b, es), rc = range_of(c, fs.c, es);
  const Range rw{static_cast<const char*>(ws), static_cast<const char*>(ws) + ws_bytes};
  if (overlap(rc, ra) || overlap(rc, rb) || overlap(rw, ra) || overlap(rw, rb) || overlap(rw, rc))
    return WP_EALIAS;

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(wp::align_up(reinterpret_cast<uintptr_t>(ws), kAlign));
  const int64_t Pa = n1 * n2, Pb = n2 * n3, Pc = n1 * n3;
  const LiftKind F = LiftKind::kForward, I = LiftKind::kInverse;
  hipError_t e = hipSuccess;
  if (gemm == WP_GEMM_NATIVE) {
    void* ah = base + pl.ah;
    void* bh = base + pl.bh;
    void* ch = base + pl.ch;
    if (dtype == WP_F64) {
      const double* A = static_cast<const double*>(a);
      const double* B = static_cast<const double*>(b);
      e = wp::launch_lift_scheme_f64(F, A, static_cast<double*>(ah), Pa, p, L, tp, s);
      if (e == hipSuccess) e = wp::launch_lift_scheme_f64(F, B, static_cast<double*>(bh), Pb, p, L, tp, s);
      if (e == hipSuccess) e = wp::launch_face_f64(static_cast<const double*>(ah), static_cast<const double*>(bh), static_cast<double*>(ch), n1, n2, n3, p, trans_a != 0, trans_b != 0, s);
      if (e == hipSuccess) e = wp::launch_lift_scheme_f64(I, static_cast<const double*>(ch), static_cast<double*>(c), Pc, p, L, tp, s);
    } else {
      const float* A = static_cast<const float*>(a);
      const float* B = static_cast<const float*>(b);
      e = wp::launch_lift_scheme_f32(F, A, static_cast<float*>(ah), Pa, p, L, tp, s);
      if (e == hipSuccess) e = wp::launch_lift_scheme_f32(F, B, static_cast<float*>(bh), Pb, p, L, tp, s);
      if (e == hipSuccess) e = wp::launch_face_f32(static_cast<const float*>(ah), static_cast<const float*>(bh), static_cast<float*>(ch), n1, n2, n3, p, trans_a != 0, trans_b != 0, s);
      if (e == hipSuccess) e = wp::launch_lift_scheme_f32(I, static_cast<const float*>(ch), static_cast<float*>(c), Pc, p, L, tp, s);
    }
  } else {
    const bool x3 = gemm == WP_GEMM_BF16X3;
    uint16_t* ahi = reinterpret_cast<uint16_t*>(base + pl.ah);
    uint16_t* alo = x3 ? reinterpret_cast<uint16_t*>(base + pl.ah_lo) : nullptr;
    uint16_t* bhi = reinterpret_cast<uint16_t*>(base + pl.bh);
    uint16_t* blo = x3 ? reinterpret_cast<uint16_t*>(base + pl.bh_lo) : nullptr;
    float* ch = reinterpret_cast<float*>(base + pl.ch);
    e = wp::launch_lift_scheme_f32_split(F, static_cast<const float*>(a), ahi, alo, Pa, p, L, tp, s);
    if (e == hipSuccess) e = wp::launch_lift_scheme_f32_split(F, static_cast<const float*>(b), bhi, blo, Pb, p, L, tp, s);
    if (e == hipSuccess) e = wp::launch_face_bf16(ahi, alo, bhi, blo, ch, n1, n2, n3, p, trans_a != 0, trans_b != 0, x3, s);
    if (e == hipSuccess) e = wp::launch_lift_scheme_f32(I, ch, static_cast<float*>(c), Pc, p, L, tp, s);
  }
  return from_hip(e);
}

}  // extern "C"

namespace {

// Shared checks of w_svd and w_svd_sparse; nsl is the number of slices the
// factors and info hold.
wp_status check_svd(int64_t n1, int64_t n2, int64_t p, int L, int k, bool sparse, int dtype,
                    int64_t* elems, int64_t* nsl) {
  if (!valid_dtype(dtype)) return WP_EDTYPE;
  const wp_status st = check_tensor(n1, n2, p, L, elems);
  if (st != WP_OK) return st;
  if (sparse && L < 1) return WP_EINVAL;
  if (k < 1 || k > n1 || k > n2 || n1 > 2048 || n2 > 2048) return WP_EINVAL;
  *nsl = sparse ? 2 * (p >> L) : p;
  return WP_OK;
}

wp_status run_svd_entry(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                        bool sparse, void* uhat, void* shat, void* vhat, void* ak,
                        int max_sweeps, int32_t* info, double* orth_err, int dtype, void* ws,
                        size_t ws_bytes, void* stream, void* ev_begin = nullptr,
                        void* ev_end = nullptr) {
  int64_t elems = 0, nsl = 0;
  const wp_status st = check_svd(n1, n2, p, L, k, sparse, dtype, &elems, &nsl);
  if (st != WP_OK) return st;
  if (a == nullptr || uhat == nullptr || shat == nullptr || vhat == nullptr || info == nullptr ||
      ws == nullptr)
    return WP_ENULL;
  const size_t need = wp::svd_workspace_bytes(n1, n2, p, L, k, sparse, dtype);
  if (ws_bytes < need) return WP_EWORKSPACE;
  const size_t es = dtype_size(dtype);
  const Range ra = range_of(a, elems, es);
  const Range outs[] = {range_of(uhat, nsl * n1 * k, es), range_of(shat, nsl * k, es),
                        range_of(vhat, nsl * n2 * k, es), range_of(ak, ak ? elems : 0, es),
                        range_of(info, nsl, 4), range_of(orth_err, orth_err ? 2 : 0, 8),
                        Range{static_cast<const char*>(ws), static_cast<const char*>(ws) + ws_bytes}};
  constexpr int nout = sizeof(outs) / sizeof(outs[0]);
  for (int i = 0; i < nout; ++i) {
    if (overlap(outs[i], ra)) return WP_EALIAS;
    for (int j = i + 1; j < nout; ++j)
      if (overlap(outs[i], outs[j])) return WP_EALIAS;
  }
  return from_hip(wp::launch_svd(a, n1, n2, p, L, k, sparse, uhat, shat, vhat, ak, max_sweeps,
                                 info, orth_err, dtype, ws, static_cast<hipStream_t>(stream),
                                 static_cast<hipEvent_t>(ev_begin), static_cast<hipEvent_t>(ev_end)));
}

}  // namespace

extern "C" {

size_t w_svd_workspace(int64_t n1, int64_t n2, int64_t p, int L, int k, int dtype) {
  int64_t elems = 0, nsl = 0;
  if (check_svd(n1, n2, p, L, k, false, dtype, &elems, &nsl) != WP_OK) return 0;
  return wp::svd_workspace_bytes(n1, n2, p, L, k, false, dtype);
}

wp_status w_svd(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k, void* uhat,
                void* shat, void* vhat, void* ak, int max_sweeps, int32_t* info, double* orth_err,
                int dtype, void* ws, size_t ws_bytes, void* stream) {
  return run_svd_entry(a, n1, n2, p, L, k, false, uhat, shat, vhat, ak, max_sweeps, info,
                       orth_err, dtype, ws, ws_bytes, stream);
}

wp_status w_svd_timed(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                      void* uhat, void* shat, void* vhat, void* ak, int max_sweeps,
                      int32_t* info, double* orth_err, int dtype, void* ws, size_t ws_bytes,
                      void* stream, void* jacobi_begin, void* jacobi_end) {
  return run_svd_entry(a, n1, n2, p, L, k, false, uhat, shat, vhat, ak, max_sweeps, info,
                       orth_err, dtype, ws, ws_bytes, stream, jacobi_begin, jacobi_end);
}

size_t w_svd_sparse_workspace(int64_t n1, int64_t n2, int64_t p, int L, int k, int dtype) {
  int64_t elems = 0, nsl = 0;
  if (check_svd(n1, n2, p, L, k, true, dtype, &elems, &nsl) != WP_OK) return 0;
  return wp::svd_workspace_bytes(n1, n2, p, L, k, true, dtype);
}

wp_status w_svd_sparse(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                       void* uhat, void* shat, void* vhat, void* ak, int max_sweeps,
                       int32_t* info, double* orth_err, int dtype, void* ws, size_t ws_bytes,
                       void* stream) {
  return run_svd_entry(a, n1, n2, p, L, k, true, uhat, shat, vhat, ak, max_sweeps, info,
                       orth_err, dtype, ws, ws_bytes, stream);
}

size_t w_pinv_workspace(int64_t n1, int64_t n2, int64_t p, int L, int sparse, int dtype) {
  int64_t elems = 0, nsl = 0;
  const int k = int(n1 < n2 ? n1 : n2);
  if (check_svd(n1, n2, p, L, k < 1 ? 1 : k, sparse != 0, dtype, &elems, &nsl) != WP_OK) return 0;
  return wp::pinv_workspace_bytes(n1, n2, p, L, sparse != 0, dtype);
}

wp_status w_pinv(const void* a, void* out, int64_t n1, int64_t n2, int64_t p, int L, int sparse,
                 double rtol, int32_t* info, int dtype, void* ws, size_t ws_bytes, void* stream) {
  int64_t elems = 0, nsl = 0;
  const int k = int(n1 < n2 ? n1 : n2);
  const wp_status st = check_svd(n1, n2, p, L, k < 1 ? 1 : k, sparse != 0, dtype, &elems, &nsl);
  if (st != WP_OK) return st;
  if (!(rtol >= 0.0) || rtol >= 1.0) return WP_EINVAL;  // also rejects NaN
  if (a == nullptr || out == nullptr || info == nullptr || ws == nullptr) return WP_ENULL;
  const size_t need = wp::pinv_workspace_bytes(n1, n2, p, L, sparse != 0, dtype);
  if (ws_bytes < need) return WP_EWORKSPACE;
  const size_t es = dtype_size(dtype);
  const Range ra = range_of(a, elems, es);
  const Range outs[] = {range_of(out, elems, es), range_of(info, nsl, 4),
                        Range{static_cast<const char*>(ws), static_cast<const char*>(ws) + ws_bytes}};
  constexpr int nout = sizeof(outs) / sizeof(outs[0]);
  for (int i = 0; i < nout; ++i) {
    if (overlap(outs[i], ra)) return WP_EALIAS;
    for (int j = i + 1; j < nout; ++j)
      if (overlap(outs[i], outs[j])) return WP_EALIAS;
  }
  if (rtol == 0.0) rtol = double(n1 > n2 ? n1 : n2) * (dtype == WP_F64 ? 2.220446049250313e-16
                                                                       : 1.1920928955078125e-07);
  return from_hip(wp::launch_pinv(a, out, n1, n2, p, L, sparse != 0, rtol, info, dtype, ws,
                                  static_cast<hipStream_t>(stream)));
}

}  // extern "C"
