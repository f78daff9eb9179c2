// Face-product GEMMs on MFMA for gfx950: C[k] = op(A[k]) op(B[k]) for every
// coefficient slice k (Def. 2.1, Alg. 1 middle part).
//
// One templated kernel serves the three arithmetic families:
//   FP64  : v_mfma_f64_16x16x4f64,   64 x 64 workgroup tile, BK = 8
//   FP32  : v_mfma_f32_32x32x2f32,  128 x 128 workgroup tile, BK = 16
//   BF16  : v_mfma_f32_32x32x16_bf16, 256 x 256 workgroup tile, BK = 32, with
//           the split-precision variant hi*hi + hi*lo + lo*hi accumulated in
//           FP32 (the lo*lo term is dropped).
// A workgroup is a WM x WN grid of wavefronts (2 x 2; 2 x 4 for BF16, two per SIMD).  Operand tiles are staged in LDS
// with K contiguous inside each row, so every lane fetches one 16-byte chunk of
// consecutive-K values per fragment read (one ds_read_b128).  Rows are 64 B
// (4 chunks) and chunk c of row r is stored at chunk c ^ ((r >> 1) & 3), which
// makes the 16-byte reads of 8 consecutive rows hit disjoint banks.  Operands
// stored with K as the slow dimension (A transposed, B not transposed) are
// transposed in registers on their way to LDS: a thread loads a CH x RW
// micro-block (RW = CH, or 4 for bf16) with CH loads and writes RW 16-byte
// LDS chunks.
//
// Pipeline: two LDS stages; the global loads of tile t+1 are issued into
// registers before the MFMAs of tile t and written to the other stage after
// them, so one barrier per K-tile suffices.
//
// Tile order: the hardware deals workgroups round-robin over the 8 XCDs; the
// linear id is remapped so that consecutive logical tiles - the tiles of one
// slice, which share A rows and B columns - land on the same XCD and its L2.

#include "wp_internal.h"

namespace wp {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kChunksPerRow = 4;  // 64-byte LDS rows
constexpr int kNumXcd = 8;

struct CfgF64 {
  using In = double;
  using Out = double;
  using Acc = f64x4;
  static constexpr int CH = 2;     // elements per 16-byte chunk
  static constexpr int TM = 16;    // MFMA tile edge
  static constexpr int G = 4;      // lane groups per MFMA (64 / TM)
  static constexpr int MT = 2;     // MFMA tiles per wave along M
  static constexpr int NT = 2;     // MFMA tiles per wave along N
  static constexpr int WM = 2;     // wavefronts along M
  static constexpr int WN = 2;     // wavefronts along N
  static constexpr int ACC_REGS = 4;
  static constexpr bool kSplit = false;
};

struct CfgF32 {
  using In = float;
  using Out = float;
  using Acc = f32x16;
  static constexpr int CH = 4;
  static constexpr int TM = 32;
  static constexpr int G = 2;
  static constexpr int MT = 2;
  static constexpr int NT = 2;
  static constexpr int WM = 2;
  static constexpr int WN = 2;
  static constexpr int ACC_REGS = 16;
  static constexpr bool kSplit = false;
};

struct CfgBF16 {
  using In = uint16_t;
  using Out = float;
  using Acc = f32x16;
  static constexpr int CH = 8;
  static constexpr int TM = 32;
  static constexpr int G = 2;
  static constexpr int MT = 4;
  static constexpr int NT = 2;
  static constexpr int WM = 2;     // 8 wavefronts, two per SIMD: one computes while
  static constexpr int WN = 4;     // the other waits on memory
  static constexpr int ACC_REGS = 16;
  static constexpr bool kSplit = true;
};

template <class Cfg>
struct Dims {
  static constexpr int BK = Cfg::CH * kChunksPerRow;        // K per LDS stage
  static constexpr int THREADS = 64 * Cfg::WM * Cfg::WN;
  static constexpr int BM = Cfg::WM * Cfg::MT * Cfg::TM;
  static constexpr int BN = Cfg::WN * Cfg::NT * Cfg::TM;
  static constexpr int KG = kChunksPerRow / Cfg::G;          // k-groups per stage
  static constexpr int ROW_BYTES = 16 * kChunksPerRow;
  static constexpr int A_BYTES = BM * ROW_BYTES;
  static constexpr int B_BYTES = BN * ROW_BYTES;
  static constexpr int NPLANE = Cfg::kSplit ? 2 : 1;         // hi (+ lo)
  static constexpr int STAGE_BYTES = NPLANE * (A_BYTES + B_BYTES);
  static constexpr int LDS_BYTES = 2 * STAGE_BYTES;
};

// Reads of 8 consecutive rows (MFMA fragments) stay conflict-free through the
// (row >> 1) term; the (row >> 3) term spreads the transposed-path writes, in
// which the lanes of a wave write rows 8 apart.
__device__ __forceinline__ int swz_chunk(int row, int c) { return c ^ (((row >> 1) ^ (row >> 3)) & 3); }

__device__ __forceinline__ int lds_off(int row, int c) {
  return row * (16 * kChunksPerRow) + swz_chunk(row, c) * 16;
}

// ---- MFMA wrappers ---------------------------------------------------------
__device__ __forceinline__ void mma(const CfgF64&, const u32x4& a, const u32x4& b, f64x4& c) {
  double av[2], bv[2];
  __builtin_memcpy(av, &a, 16);
  __builtin_memcpy(bv, &b, 16);
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bv[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bv[1], c, 0, 0, 0);
}

__device__ __forceinline__ void mma(const CfgF32&, const u32x4& a, const u32x4& b, f32x16& c) {
  float av[4], bv[4];
  __builtin_memcpy(av, &a, 16);
  __builtin_memcpy(bv, &b, 16);
#pragma unroll
  for (int i = 0; i < 4; ++i) c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[i], c, 0, 0, 0);
}

__device__ __forceinline__ void mma_bf16(const u32x4& a, const u32x4& b, f32x16& c) {
  bf16x8 av, bv;
  __builtin_memcpy(&av, &a, 16);
  __builtin_memcpy(&bv, &b, 16);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
}

// ---- global -> register staging -------------------------------------------
// One operand tile in NPL planes (hi, and lo for the split products): R rows
// (M or N) by BK columns of K.  K_CONTIG: the stored matrix has K contiguous
// (row pitch ld along R); otherwise R is contiguous and the pitch ld runs
// along K.  The work items of all planes are dealt over the whole workgroup.
template <class Cfg, int R, bool K_CONTIG, int NPL, int kThreads>
struct TileLoader {
  using In = typename Cfg::In;
  static constexpr int CH = Cfg::CH;
  static constexpr int BK = CH * kChunksPerRow;
  // Transposed staging: micro-blocks of CH K-rows by RW R-columns (RW = 4 for
  // bf16, i.e. 8-byte loads, to keep the staged block at 16 registers).
  static constexpr int RW = CH == 8 ? 4 : CH;
  static constexpr int LB = RW * int(sizeof(In));  // bytes per transposed-path load
  // Work items per plane: K-contiguous -> one chunk each; otherwise one
  // CH x RW micro-block each.
  static constexpr int ITEMS = K_CONTIG ? R * kChunksPerRow : (BK / CH) * (R / RW);
  static constexpr int TOTAL = ITEMS * NPL;
  static constexpr int PER_THREAD = (TOTAL + kThreads - 1) / kThreads;
  static constexpr int WORDS = K_CONTIG ? 4 : CH * LB / 4;  // 32-bit words per item
  unsigned int buf[PER_THREAD][WORDS];

  // Load element (r, k) of the tile with bounds checks (zero outside).
  __device__ __forceinline__ static In elem(const In* base, int64_t ld, int r, int k, int rlim,
                                            int klim) {
    if (r >= rlim || k >= klim) return In(0);
    return K_CONTIG ? base[int64_t(r) * ld + k] : base[int64_t(k) * ld + r];
  }

  // base[p] points at element (row 0, k 0) of plane p; rlim/klim = rows/K left.
  __device__ __forceinline__ void load(const In* const* base, int64_t ld, int rlim, int klim,
                                       bool vec_ok) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int all = tid + i * kThreads;
      if (TOTAL % kThreads != 0 && all >= TOTAL) break;
      const int plane = NPL == 1 ? 0 : all / ITEMS;
      const int item = NPL == 1 ? all : all % ITEMS;
      const In* b = base[plane];
      if constexpr (K_CONTIG) {
        const int r = item / kChunksPerRow;
        const int c = item % kChunksPerRow;
        const int k0 = c * CH;
        if (vec_ok && r < rlim && k0 + CH <= klim) {
          const u32x4 v = *reinterpret_cast<const u32x4*>(b + int64_t(r) * ld + k0);
          __builtin_memcpy(&buf[i][0], &v, 16);
        } else {
          In tmp[CH];
#pragma unroll
          for (int e = 0; e < CH; ++e) tmp[e] = elem(b, ld, r, k0 + e, rlim, klim);
          __builtin_memcpy(&buf[i][0], tmp, 16);
        }
      } else {
        constexpr int RB = R / RW;  // micro-blocks along R
        const int kb = item / RB;
        const int rb = item % RB;
        const int k0 = kb * CH;
        const int r0 = rb * RW;
#pragma unroll
        for (int e = 0; e < CH; ++e) {
          const int k = k0 + e;
          unsigned int* dst = &buf[i][e * (LB / 4)];
          if (vec_ok && k < klim && r0 + RW <= rlim) {
            if constexpr (LB == 16) {
              const u32x4 v = *reinterpret_cast<const u32x4*>(b + int64_t(k) * ld + r0);
              __builtin_memcpy(dst, &v, 16);
            } else {
              const u32x2 v = *reinterpret_cast<const u32x2*>(b + int64_t(k) * ld + r0);
              __builtin_memcpy(dst, &v, 8);
            }
          } else {
            In tmp[RW];
#pragma unroll
            for (int f = 0; f < RW; ++f) tmp[f] = elem(b, ld, r0 + f, k, rlim, klim);
            __builtin_memcpy(dst, tmp, LB);
          }
        }
      }
    }
  }

  // Write the staged items into the LDS planes (rows of BK K-values); plane p
  // starts plane_bytes * p after lds.
  __device__ __forceinline__ void store(char* __restrict__ lds, int plane_bytes) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int all = tid + i * kThreads;
      if (TOTAL % kThreads != 0 && all >= TOTAL) break;
      const int plane = NPL == 1 ? 0 : all / ITEMS;
      const int item = NPL == 1 ? all : all % ITEMS;
      char* dst = lds + plane * plane_bytes;
      if constexpr (K_CONTIG) {
        const int r = item / kChunksPerRow;
        const int c = item % kChunksPerRow;
        u32x4 v;
        __builtin_memcpy(&v, &buf[i][0], 16);
        *reinterpret_cast<u32x4*>(dst + lds_off(r, c)) = v;
      } else {
        constexpr int RB = R / RW;
        const int kb = item / RB;
        const int rb = item % RB;
        const int r0 = rb * RW;
        // buf[i] holds K-rows k0..k0+CH-1 of R-columns r0..r0+RW-1; emit R-row
        // r0+f holding K-values k0..k0+CH-1 (chunk index kb).
        In m[CH][RW];
        __builtin_memcpy(m, &buf[i][0], CH * LB);
#pragma unroll
        for (int f = 0; f < RW; ++f) {
          In col[CH];
#pragma unroll
          for (int e = 0; e < CH; ++e) col[e] = m[e][f];
          u32x4 v;
          __builtin_memcpy(&v, col, 16);
          *reinterpret_cast<u32x4*>(dst + lds_off(r0 + f, kb)) = v;
        }
      }
    }
  }
};

// Map the hardware workgroup id to a logical tile id so that runs of
// consecutive logical ids stay on one XCD.
__device__ __forceinline__ int64_t xcd_remap(int64_t hw, int64_t total) {
  const int64_t xcd = hw % kNumXcd;
  const int64_t j = hw / kNumXcd;
  const int64_t q = total / kNumXcd;
  const int64_t r = total % kNumXcd;
  return xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
}

struct GemmArgs {
  const void* a_hi;
  const void* a_lo;
  const void* b_hi;
  const void* b_lo;
  void* c;
  int m, n, k;
  int64_t lda, ldb, ldc;        // row pitch of the stored matrices
  int64_t sa, sb, sc;           // slice strides (elements)
  int64_t batch;
  int tiles_m, tiles_n;
  int vec_a, vec_b;             // 16-byte global loads allowed
};

template <class Cfg, bool TA, bool TB, bool X3>
__global__ __launch_bounds__(64 * Cfg::WM * Cfg::WN, 1) void face_gemm_kernel(GemmArgs args) {
  using In = typename Cfg::In;
  using Out = typename Cfg::Out;
  using Acc = typename Cfg::Acc;
  using D = Dims<Cfg>;
  constexpr int BM = D::BM, BN = D::BN, BK = D::BK;
  constexpr int TM = Cfg::TM, G = Cfg::G, MT = Cfg::MT, NT = Cfg::NT;
  constexpr bool SPLIT = Cfg::kSplit;
  constexpr bool USE_LO = SPLIT && X3;

  extern __shared__ __align__(16) char smem[];

  const int64_t tiles_per_slice = int64_t(args.tiles_m) * args.tiles_n;
  const int64_t total = tiles_per_slice * args.batch;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t slice = logical / tiles_per_slice;
  const int64_t t_in = logical % tiles_per_slice;
  const int tm = int(t_in / args.tiles_n);
  const int tn = int(t_in % args.tiles_n);
  const int m0 = tm * BM;
  const int n0 = tn * BN;

  const In* a_hi = static_cast<const In*>(args.a_hi) + slice * args.sa;
  const In* b_hi = static_cast<const In*>(args.b_hi) + slice * args.sb;
  const In* a_lo = USE_LO ? static_cast<const In*>(args.a_lo) + slice * args.sa : nullptr;
  const In* b_lo = USE_LO ? static_cast<const In*>(args.b_lo) + slice * args.sb : nullptr;

  // Tile origin in the stored matrices: A stored (m, k) or (k, m); B stored
  // (k, n) or (n, k).
  auto a_origin = [&](const In* base, int k0) {
    return TA ? base + int64_t(k0) * args.lda + m0 : base + int64_t(m0) * args.lda + k0;
  };
  auto b_origin = [&](const In* base, int k0) {
    return TB ? base + int64_t(n0) * args.ldb + k0 : base + int64_t(k0) * args.ldb + n0;
  };

  constexpr int NPL = USE_LO ? 2 : 1;
  TileLoader<Cfg, BM, !TA, NPL, D::THREADS> la;
  TileLoader<Cfg, BN, TB, NPL, D::THREADS> lb;

  const int rlim_a = args.m - m0;
  const int rlim_b = args.n - n0;
  const bool va = args.vec_a != 0;
  const bool vb = args.vec_b != 0;

  // LDS stage layout: A hi | A lo | B hi | B lo (lo planes only for bf16x3).
  constexpr int A_PLANES = D::A_BYTES * NPL;
  auto issue_loads = [&](int k0) {
    const int klim = args.k - k0;
    const In* pa[2] = {a_origin(a_hi, k0), USE_LO ? a_origin(a_lo, k0) : nullptr};
    const In* pb[2] = {b_origin(b_hi, k0), USE_LO ? b_origin(b_lo, k0) : nullptr};
    la.load(pa, args.lda, rlim_a, klim, va);
    lb.load(pb, args.ldb, rlim_b, klim, vb);
  };
  auto stage_ptr = [&](int stage) { return smem + stage * D::STAGE_BYTES; };
  auto commit = [&](int stage) {
    char* s = stage_ptr(stage);
    la.store(s, D::A_BYTES);
    lb.store(s + A_PLANES, D::B_BYTES);
  };

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave / Cfg::WN) * (MT * TM);  // wave origin inside the tile
  const int wn = (wave % Cfg::WN) * (NT * TM);
  const int lrow = lane % TM;
  const int lgrp = lane / TM;

  Acc acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < Cfg::ACC_REGS; ++r) acc[i][j][r] = 0;

  const int nk = (args.k + BK - 1) / BK;
  issue_loads(0);
  commit(0);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) issue_loads((kt + 1) * BK);

    const char* s = stage_ptr(cur);
    const char* sa_hi = s;
    const char* sa_lo = s + D::A_BYTES;
    const char* sb_hi = s + A_PLANES;
    const char* sb_lo = s + A_PLANES + D::B_BYTES;
#pragma unroll
    for (int kg = 0; kg < D::KG; ++kg) {
      const int c = kg * G + lgrp;
      // B fragments for the whole k-group, then one A fragment (pair) at a
      // time, so that few fragment registers are live beside the accumulators.
      u32x4 fb[NT], fb_lo[USE_LO ? NT : 1];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int off = lds_off(wn + j * TM + lrow, c);
        fb[j] = *reinterpret_cast<const u32x4*>(sb_hi + off);
        if constexpr (USE_LO) fb_lo[j] = *reinterpret_cast<const u32x4*>(sb_lo + off);
      }
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const int off = lds_off(wm + i * TM + lrow, c);
        const u32x4 fa = *reinterpret_cast<const u32x4*>(sa_hi + off);
        u32x4 fa_lo;
        if constexpr (USE_LO) fa_lo = *reinterpret_cast<const u32x4*>(sa_lo + off);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          if constexpr (SPLIT) {
            if constexpr (USE_LO) {
              mma_bf16(fa_lo, fb[j], acc[i][j]);
              mma_bf16(fa, fb_lo[j], acc[i][j]);
            }
            mma_bf16(fa, fb[j], acc[i][j]);
          } else {
            mma(Cfg{}, fa, fb[j], acc[i][j]);
          }
        }
      }
    }

    if (kt + 1 < nk) commit(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: MFMA output layout.  32x32 FP32-accumulator tiles: register r of
  // lane l holds row (r/4)*8 + (l/32)*4 + r%4, column l%32.  16x16 FP64 tiles:
  // register r of lane l holds row 4*r + l/16, column l%16.
  Out* cbase = static_cast<Out*>(args.c) + slice * args.sc;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = n0 + wn + j * TM + lrow;
#pragma unroll
      for (int r = 0; r < Cfg::ACC_REGS; ++r) {
        const int rr = (TM == 32) ? ((r / 4) * 8 + lgrp * 4 + (r % 4)) : (r * 4 + lgrp);
        const int row = m0 + wm + i * TM + rr;
        if (row < args.m && col < args.n) cbase[int64_t(row) * args.ldc + col] = Out(acc[i][j][r]);
      }
    }
}

template <class Cfg, bool TA, bool TB, bool X3>
hipError_t launch_cfg(const GemmArgs& a0, hipStream_t s) {
  using D = Dims<Cfg>;
  GemmArgs a = a0;
  a.tiles_m = int((a.m + D::BM - 1) / D::BM);
  a.tiles_n = int((a.n + D::BN - 1) / D::BN);
  const int64_t total = int64_t(a.tiles_m) * a.tiles_n * a.batch;
  if (total == 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidConfiguration;
  auto kern = face_gemm_kernel<Cfg, TA, TB, X3>;
  static bool attr_set = false;  // per instantiation; setting it twice is harmless
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, D::LDS_BYTES);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(unsigned(total)), dim3(D::THREADS), D::LDS_BYTES, s, a);
  return hipGetLastError();
}

template <class Cfg, bool X3>
hipError_t dispatch(const GemmArgs& a, bool ta, bool tb, hipStream_t s) {
  if (!ta && !tb) return launch_cfg<Cfg, false, false, X3>(a, s);
  if (ta && !tb) return launch_cfg<Cfg, true, false, X3>(a, s);
  if (!ta && tb) return launch_cfg<Cfg, false, true, X3>(a, s);
  return launch_cfg<Cfg, true, true, X3>(a, s);
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <class Cfg>
GemmArgs make_args(const void* ahi, const void* alo, const void* bhi, const void* blo, void* c,
                   int64_t m, int64_t kk, int64_t n, int64_t batch, bool ta, bool tb) {
  constexpr int CH = Cfg::CH;
  GemmArgs a{};
  a.a_hi = ahi;
  a.a_lo = alo;
  a.b_hi = bhi;
  a.b_lo = blo;
  a.c = c;
  a.m = int(m);
  a.n = int(n);
  a.k = int(kk);
  a.lda = ta ? m : kk;
  a.ldb = tb ? kk : n;
  a.ldc = n;
  a.sa = m * kk;
  a.sb = kk * n;
  a.sc = m * n;
  a.batch = batch;
  // 16-byte loads need 16-byte aligned rows: pitch and slice stride multiples
  // of a chunk and aligned base pointers.
  a.vec_a = (a.lda % CH == 0) && (a.sa % CH == 0) && aligned16(ahi) && (alo == nullptr || aligned16(alo));
  a.vec_b = (a.ldb % CH == 0) && (a.sb % CH == 0) && aligned16(bhi) && (blo == nullptr || aligned16(blo));
  return a;
}

}  // namespace

hipError_t launch_face_f64(const double* a, const double* b, double* c, int64_t m, int64_t kk,
                           int64_t n, int64_t batch, bool ta, bool tb, hipStream_t s) {
  return dispatch<CfgF64, false>(make_args<CfgF64>(a, nullptr, b, nullptr, c, m, kk, n, batch, ta, tb),
                                 ta, tb, s);
}

hipError_t launch_face_f32(const float* a, const float* b, float* c, int64_t m, int64_t kk,
                           int64_t n, int64_t batch, bool ta, bool tb, hipStream_t s) {
  return dispatch<CfgF32, false>(make_args<CfgF32>(a, nullptr, b, nullptr, c, m, kk, n, batch, ta, tb),
                                 ta, tb, s);
}

hipError_t launch_face_bf16(const uint16_t* ahi, const uint16_t* alo, const uint16_t* bhi,
                            const uint16_t* blo, float* c, int64_t m, int64_t kk, int64_t n,
                            int64_t batch, bool ta, bool tb, bool x3, hipStream_t s) {
  const GemmArgs a = make_args<CfgBF16>(ahi, x3 ? alo : nullptr, bhi, x3 ? blo : nullptr, c, m, kk,
                                        n, batch, ta, tb);
  return x3 ? dispatch<CfgBF16, true>(a, ta, tb, s) : dispatch<CfgBF16, false>(a, ta, tb, s);
}

}  // namespace wp
