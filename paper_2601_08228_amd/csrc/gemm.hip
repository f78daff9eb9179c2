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
// BF16 operands whose dimensions allow whole 16-byte chunks (the common case)
// take a second kernel, face_bf16_direct, whose copies go from global memory
// straight into LDS (buffer_load ... lds) through a ring of K stages, with
// transposed operands read by ds_read_b64_tr_b16; see its description below.
//
// Tile order: the hardware deals workgroups round-robin over the 8 XCDs; the
// linear id is remapped so that consecutive logical tiles - the tiles of one
// slice, which share A rows and B columns - land on the same XCD and its L2.

#include <type_traits>

#include <atomic>

#include "wp_internal.h"

namespace wp {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for_n(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for_n<N, I + 1>(f);
  }
}

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

// ---- BF16 face-product with direct-to-LDS loads -----------------------------
// The global -> LDS copies bypass registers (buffer_load ... lds, 16 bytes per
// lane), so several K stages can be in flight: stage t is consumed while
// stages t+1 .. t+S-1 load.  Each operand keeps its stored layout in LDS:
//   * K contiguous in memory ("KC": A not transposed, B transposed): LDS rows
//     of BK = 32 K values (64 bytes, one global load of 4 lanes per row);
//     chunk c (8 values) of row r sits at chunk c ^ ((r >> 2) & 3), so the
//     fragment reads of 8 or 16 consecutive rows cover disjoint banks;
//   * K slow in memory ("KS"): LDS rows are the 32 K values' rows of 256
//     elements (512 bytes); chunk c of K-row k sits at c ^ h(k), h(k) = 0, 6,
//     10, 12 for k mod 4 = 0..3; fragments are read with ds_read_b64_tr_b16,
//     which hands lane j of each 16-lane group element [k0 + q][r0 + j]
//     (q = 0..3) when lane i addresses [k0 + i/4][r0 + 4 (i mod 4)].
// A stage holds two MFMA K steps of 16; each plane is filled by two copies per
// lane (rows 0-127 and 128-255, or K-rows 0-15 and 16-31), 8 KiB each.
// Lanes outside the matrix get an offset past the buffer's end, so the
// hardware returns zeros for them.
namespace dl {
constexpr int BM = 256, BN = 256, BK = 32, TM = 32;
constexpr int WN = 4, MT = 4, NT = 2;
constexpr int THREADS = 512;
constexpr int PLANE = 256 * BK * 2;  // bytes of one operand plane of one stage
constexpr uint32_t kOut = 0x80000000u;  // buffer offset that reads as zero
}  // namespace dl

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_t;

__device__ __forceinline__ int kc_chunk(int row, int c) { return c ^ ((row >> 2) & 3); }
__device__ __forceinline__ int ks_h(int k) { return (0x0C0A0600 >> (8 * (k & 3))) & 0xFF; }

// s_waitcnt with only the vector-memory counter limited to n (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt and lgkmcnt left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt((N & 15) | (((N >> 4) & 3) << 14) | (7 << 4) | (15 << 8));
}
// Wait until at most `stages` stages of LPS loads each are pending (stages <= S - 2).
template <int S, int LPS>
__device__ __forceinline__ void wait_stages(int stages) {
  static_for_n<S - 1>([&](auto I) {
    constexpr int P = decltype(I)::value;
    if (stages == P) wait_vm<P * LPS>();
  });
}

// 32-bit LDS address of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return static_cast<uint32_t>(
      reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char*)p));
}

// Per-lane source geometry of one operand plane (see the layouts above).
struct DlSrc {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t base;     // byte offset of this lane's chunk at k0 = 0
  uint32_t kstep;    // bytes per K element of k0
  int kidx;          // K index of this lane's chunk relative to k0 (KC: 8c, KS: k)
  bool rok;          // the lane's rows / columns are inside the matrix
};

template <bool KC>
__device__ __forceinline__ DlSrc dl_src(const uint16_t* plane, int64_t ld, int r0, int rtot,
                                        int kk, int i) {
  DlSrc d;
  const int t = threadIdx.x;
  if constexpr (KC) {
    const int r = (t >> 2) + 128 * i;
    const int c = kc_chunk(r, t & 3);
    d.base = uint32_t(((int64_t(r0) + r) * ld + 8 * c) * 2);
    d.kstep = 2;
    d.kidx = 8 * c;
    d.rok = r0 + r < rtot;
    d.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(plane), 0,
                                               int(int64_t(rtot) * ld * 2), 0x00020000);
  } else {
    const int k = (t >> 5) + 16 * i;
    const int c = (t & 31) ^ ks_h(k);
    d.base = uint32_t((int64_t(k) * ld + r0 + 8 * c) * 2);
    d.kstep = uint32_t(ld * 2);
    d.kidx = k;
    d.rok = r0 + 8 * c < rtot;
    d.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(plane), 0,
                                               int(int64_t(kk) * ld * 2), 0x00020000);
  }
  return d;
}

__device__ __forceinline__ void dl_issue(const DlSrc& d, char* lds_plane, int k0, int kk) {
  // (lds_plane: the 8 KiB half of the plane that this copy fills)
  const bool ok = d.rok && (k0 + d.kidx < kk);
  const uint32_t off = ok ? d.base + uint32_t(k0) * d.kstep : dl::kOut;
  // Each wavefront fills 1 KiB of the plane: lane l writes bytes 16 l of it.
  // (The pointer stays derived from the stage buffer, so the compiler knows
  // which LDS object the copy writes.)
  const int wave_off = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x & ~63) * 16);
  __attribute__((address_space(3))) char* dst = (__attribute__((address_space(3))) char*)lds_plane;
  __builtin_amdgcn_raw_ptr_buffer_load_lds(d.rsrc, (lds_t*)(dst + wave_off), 16, off, 0, 0, 0);
}

// ---- fragment reads ----------------------------------------------------------
// The LDS reads of a stage are written as inline assembly, each block ending
// with its own lgkmcnt(0) wait: the compiler cannot tell which LDS object a
// buffer-to-LDS copy writes, so for reads it can see it would wait for every
// copy in flight (vmcnt(0)), which would undo the multi-stage pipeline.  The
// copies a stage depends on are waited for explicitly before the barrier.
// The outputs are early-clobber: a read's data can land while later reads of
// the same block still need their address registers.

// Per-lane byte offset, inside a stage buffer, of the lane's 16-byte K-chunk of
// tile row xb + (l & 31) in a K-contiguous plane (MFMA operand layout: K
// values 8 (l >> 5) .. +7 of the stage's first K step; the second step's
// chunk is two further, at this offset ^ 32).  Tiles 32 rows apart differ by
// 2048 bytes.
__device__ __forceinline__ uint32_t kc_lane_off() {
  const int l = threadIdx.x & 63;
  const int row = l & 31;
  return uint32_t(row * (dl::BK * 2) + 16 * kc_chunk(row, l >> 5));
}

// Per-lane byte offset of a K-slow plane's transposed read: lane i of 16-lane
// group g addresses K-row 8 (g >> 1) + 4 half + i / 4, columns
// xb + 16 (g & 1) + 4 (i mod 4) .. +3 (the stage's second K step: 16 K-rows,
// 8 KiB, further).
__device__ __forceinline__ uint32_t ks_lane_off(int xb, int half) {
  const int l = threadIdx.x & 63;
  const int g = l >> 4, i = l & 15;
  const int r = xb + 16 * (g & 1) + 4 * (i & 3);
  const int k = 8 * (g >> 1) + 4 * half + (i >> 2);
  return uint32_t(k * (dl::BM * 2) + 16 * ((r >> 3) ^ ks_h(k)) + 8 * (i & 1));
}

// K-contiguous fragments: T tiles (32 rows apart) of NPL planes (16 KiB apart).
template <int T, int NPL>
__device__ __forceinline__ void kc_frags(uint32_t a, u32x4 (&f)[T * NPL]) {
  if constexpr (T == 2 && NPL == 1) {
    asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:2048\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(f[0]), "=&v"(f[1]) : "v"(a) : "memory");
  } else if constexpr (T == 2 && NPL == 2) {
    asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %4 offset:2048\n\t"
                 "ds_read_b128 %2, %4 offset:16384\n\tds_read_b128 %3, %4 offset:18432\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(f[0]), "=&v"(f[1]), "=&v"(f[2]), "=&v"(f[3]) : "v"(a) : "memory");
  } else if constexpr (T == 4 && NPL == 1) {
    asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %4 offset:2048\n\t"
                 "ds_read_b128 %2, %4 offset:4096\n\tds_read_b128 %3, %4 offset:6144\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(f[0]), "=&v"(f[1]), "=&v"(f[2]), "=&v"(f[3]) : "v"(a) : "memory");
  } else {
    static_assert(T == 4 && NPL == 2, "unsupported fragment count");
    asm volatile("ds_read_b128 %0, %8\n\tds_read_b128 %1, %8 offset:2048\n\t"
                 "ds_read_b128 %2, %8 offset:4096\n\tds_read_b128 %3, %8 offset:6144\n\t"
                 "ds_read_b128 %4, %8 offset:16384\n\tds_read_b128 %5, %8 offset:18432\n\t"
                 "ds_read_b128 %6, %8 offset:20480\n\tds_read_b128 %7, %8 offset:22528\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(f[0]), "=&v"(f[1]), "=&v"(f[2]), "=&v"(f[3]), "=&v"(f[4]), "=&v"(f[5]),
                   "=&v"(f[6]), "=&v"(f[7])
                 : "v"(a) : "memory");
  }
}

// K-slow fragments by transposed reads: addresses ad[2 t + half] for tile t,
// plane p at + PLANE p, all at the immediate offset OFF (the K step of the
// stage); output h[(p T + t) 2 + half] holds 4 K values.
template <int T, int NPL, int OFF>
__device__ __forceinline__ void ks_frags(const uint32_t (&ad)[2 * T], u32x2 (&h)[2 * T * NPL]) {
  if constexpr (T == 2 && NPL == 1) {
    asm volatile(
                 "ds_read_b64_tr_b16 %[h0], %[a0] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h1], %[a1] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h2], %[a2] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h3], %[a3] offset:%[o0]\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : [h0] "=&v"(h[0]), [h1] "=&v"(h[1]), [h2] "=&v"(h[2]), [h3] "=&v"(h[3])
                 : [a0] "v"(ad[0]), [a1] "v"(ad[1]), [a2] "v"(ad[2]), [a3] "v"(ad[3]), [o0] "i"(OFF), [o1] "i"(OFF + dl::PLANE) : "memory");
  } else if constexpr (T == 2 && NPL == 2) {
    asm volatile(
                 "ds_read_b64_tr_b16 %[h0], %[a0] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h1], %[a1] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h2], %[a2] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h3], %[a3] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h4], %[a0] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h5], %[a1] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h6], %[a2] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h7], %[a3] offset:%[o1]\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : [h0] "=&v"(h[0]), [h1] "=&v"(h[1]), [h2] "=&v"(h[2]), [h3] "=&v"(h[3]), [h4] "=&v"(h[4]), [h5] "=&v"(h[5]), [h6] "=&v"(h[6]), [h7] "=&v"(h[7])
                 : [a0] "v"(ad[0]), [a1] "v"(ad[1]), [a2] "v"(ad[2]), [a3] "v"(ad[3]), [o0] "i"(OFF), [o1] "i"(OFF + dl::PLANE) : "memory");
  } else if constexpr (T == 4 && NPL == 1) {
    asm volatile(
                 "ds_read_b64_tr_b16 %[h0], %[a0] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h1], %[a1] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h2], %[a2] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h3], %[a3] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h4], %[a4] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h5], %[a5] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h6], %[a6] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h7], %[a7] offset:%[o0]\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : [h0] "=&v"(h[0]), [h1] "=&v"(h[1]), [h2] "=&v"(h[2]), [h3] "=&v"(h[3]), [h4] "=&v"(h[4]), [h5] "=&v"(h[5]), [h6] "=&v"(h[6]), [h7] "=&v"(h[7])
                 : [a0] "v"(ad[0]), [a1] "v"(ad[1]), [a2] "v"(ad[2]), [a3] "v"(ad[3]), [a4] "v"(ad[4]), [a5] "v"(ad[5]), [a6] "v"(ad[6]), [a7] "v"(ad[7]), [o0] "i"(OFF), [o1] "i"(OFF + dl::PLANE) : "memory");
  } else {
    static_assert(T == 4 && NPL == 2, "unsupported fragment count");
    asm volatile(
                 "ds_read_b64_tr_b16 %[h0], %[a0] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h1], %[a1] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h2], %[a2] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h3], %[a3] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h4], %[a4] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h5], %[a5] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h6], %[a6] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h7], %[a7] offset:%[o0]\n\t"
                 "ds_read_b64_tr_b16 %[h8], %[a0] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h9], %[a1] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h10], %[a2] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h11], %[a3] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h12], %[a4] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h13], %[a5] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h14], %[a6] offset:%[o1]\n\t"
                 "ds_read_b64_tr_b16 %[h15], %[a7] offset:%[o1]\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : [h0] "=&v"(h[0]), [h1] "=&v"(h[1]), [h2] "=&v"(h[2]), [h3] "=&v"(h[3]), [h4] "=&v"(h[4]), [h5] "=&v"(h[5]), [h6] "=&v"(h[6]), [h7] "=&v"(h[7]), [h8] "=&v"(h[8]), [h9] "=&v"(h[9]), [h10] "=&v"(h[10]), [h11] "=&v"(h[11]), [h12] "=&v"(h[12]), [h13] "=&v"(h[13]), [h14] "=&v"(h[14]), [h15] "=&v"(h[15])
                 : [a0] "v"(ad[0]), [a1] "v"(ad[1]), [a2] "v"(ad[2]), [a3] "v"(ad[3]), [a4] "v"(ad[4]), [a5] "v"(ad[5]), [a6] "v"(ad[6]), [a7] "v"(ad[7]), [o0] "i"(OFF), [o1] "i"(OFF + dl::PLANE) : "memory");
  }
}

// All fragments of one operand for one stage: T tiles of NPL planes, tile t of
// plane p in f[p T + t].  KC: lane_off = kc_lane_off(); KS: ks_off[2 t + half]
// = ks_lane_off(xb + 32 t, half).
template <bool KC, int T, int NPL, int OFF>
__device__ __forceinline__ void stage_frags(uint32_t buf, uint32_t kc_off, const uint32_t (&ks_off)[2 * T],
                                            u32x4 (&f)[T * NPL]) {
  if constexpr (KC) {
    kc_frags<T, NPL>(buf + kc_off, f);
  } else {
    uint32_t ad[2 * T];
#pragma unroll
    for (int q = 0; q < 2 * T; ++q) ad[q] = buf + ks_off[q];
    u32x2 h[2 * T * NPL];
    ks_frags<T, NPL, OFF>(ad, h);
#pragma unroll
    for (int q = 0; q < T * NPL; ++q) {
      f[q][0] = h[2 * q][0];
      f[q][1] = h[2 * q][1];
      f[q][2] = h[2 * q + 1][0];
      f[q][3] = h[2 * q + 1][1];
    }
  }
}

// One LDS stage buffer per B: separate __shared__ objects, so that the
// compiler can tell the copies into one stage from the reads of another and
// only waits for the copies a read depends on.
template <int B, int BYTES>
__device__ __forceinline__ char* dl_stage() {
  __shared__ __align__(16) char buf[BYTES];
  return buf;
}

// Workgroup barrier without a memory fence: the waits for the copies are
// explicit, and the signal fences keep the compiler from moving LDS accesses
// across it.
__device__ __forceinline__ void dl_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <bool TA, bool TB, bool X3, int S>
__global__ __launch_bounds__(dl::THREADS, 1) void face_bf16_direct(GemmArgs args) {
  using namespace dl;
  constexpr int NPL = X3 ? 2 : 1;
  constexpr int STAGE = 2 * NPL * PLANE;
  constexpr bool A_KC = !TA, B_KC = TB;

  const int64_t tiles_per_slice = int64_t(args.tiles_m) * args.tiles_n;
  const int64_t total = tiles_per_slice * args.batch;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t slice = logical / tiles_per_slice;
  const int64_t t_in = logical % tiles_per_slice;
  const int m0 = int(t_in / args.tiles_n) * BM;
  const int n0 = int(t_in % args.tiles_n) * BN;
  const int kk = args.k;

  const uint16_t* pa[2] = {static_cast<const uint16_t*>(args.a_hi) + slice * args.sa,
                           X3 ? static_cast<const uint16_t*>(args.a_lo) + slice * args.sa : nullptr};
  const uint16_t* pb[2] = {static_cast<const uint16_t*>(args.b_hi) + slice * args.sb,
                           X3 ? static_cast<const uint16_t*>(args.b_lo) + slice * args.sb : nullptr};
  DlSrc sa[NPL][2], sb[NPL][2];
#pragma unroll
  for (int q = 0; q < NPL; ++q)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      sa[q][i] = dl_src<A_KC>(pa[q], args.lda, m0, args.m, kk, i);
      sb[q][i] = dl_src<B_KC>(pb[q], args.ldb, n0, args.n, kk, i);
    }
  // Copies of K stage st into stage buffer B.
  auto issue = [&](auto BB, int st) {
    char* base = dl_stage<decltype(BB)::value, STAGE>();
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        dl_issue(sa[q][i], base + q * PLANE + i * (PLANE / 2), st * BK, kk);
        dl_issue(sb[q][i], base + (NPL + q) * PLANE + i * (PLANE / 2), st * BK, kk);
      }
  };

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave / WN) * (MT * TM);
  const int wn = (wave % WN) * (NT * TM);
  const int lrow = lane % TM;
  const int lgrp = lane / TM;

  f32x16 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

  // Per-lane fragment offsets inside a stage plane (tiles 32 rows apart are
  // 1 KiB apart in a K-contiguous plane).
  const uint32_t a_kc_off = uint32_t(wm * BK * 2) + kc_lane_off();
  const uint32_t b_kc_off = uint32_t(wn * BK * 2) + kc_lane_off();
  uint32_t a_ks_off[2 * MT], b_ks_off[2 * NT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) a_ks_off[2 * t + h] = ks_lane_off(wm + 32 * t, h);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) b_ks_off[2 * t + h] = ks_lane_off(wn + 32 * t, h);

  const int nk = (kk + BK - 1) / BK;
  static_for_n<S - 1>([&](auto BB) {
    if (decltype(BB)::value < nk) issue(BB, decltype(BB)::value);
  });

  // K stage t lives in buffer t mod S; the loop is unrolled S times so that
  // every buffer index is a constant.
  for (int t0 = 0; t0 < nk; t0 += S) {
    static_for_n<S>([&](auto UU) {
      constexpr int u = decltype(UU)::value;
      const int t = t0 + u;
      if (t >= nk) return;
      // Stage t has landed once at most the stages issued after it are pending.
      const int pending = (nk - 1 < t + S - 2 ? nk - 1 : t + S - 2) - t;
      wait_stages<S, 4 * NPL>(pending);
      dl_barrier();  // every wave's copies of stage t are in LDS; stage t-1 is consumed
      if (t + S - 1 < nk) issue(std::integral_constant<int, (u + S - 1) % S>{}, t + S - 1);

      const uint32_t buf = lds_addr(dl_stage<u, STAGE>());
      // Two MFMA K steps of 16 per stage: the K-contiguous fragments of the
      // second sit at the lane offset ^ 32, the K-slow ones 16 K-rows (8 KiB)
      // further.
      static_for_n<2>([&](auto HH) {
        constexpr int h = decltype(HH)::value;
        u32x4 fa[MT * NPL], fb[NT * NPL];
        stage_frags<B_KC, NT, NPL, h * PLANE / 2>(buf + NPL * PLANE, b_kc_off ^ (32 * h), b_ks_off, fb);
        stage_frags<A_KC, MT, NPL, h * PLANE / 2>(buf, a_kc_off ^ (32 * h), a_ks_off, fa);
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            if constexpr (X3) {
              mma_bf16(fa[MT + i], fb[j], acc[i][j]);
              mma_bf16(fa[i], fb[NT + j], acc[i][j]);
            }
            mma_bf16(fa[i], fb[j], acc[i][j]);
          }
      });
    });
  }

  float* cbase = static_cast<float*>(args.c) + slice * args.sc;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = n0 + wn + j * TM + lrow;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + i * TM + (r / 4) * 8 + lgrp * 4 + (r % 4);
        if (row < args.m && col < args.n) cbase[int64_t(row) * args.ldc + col] = acc[i][j][r];
      }
    }
}

template <bool TA, bool TB, bool X3, int S>
hipError_t launch_direct(const GemmArgs& a0, hipStream_t s) {
  GemmArgs a = a0;
  a.tiles_m = int((a.m + dl::BM - 1) / dl::BM);
  a.tiles_n = int((a.n + dl::BN - 1) / dl::BN);
  const int64_t total = int64_t(a.tiles_m) * a.tiles_n * a.batch;
  if (total == 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((face_bf16_direct<TA, TB, X3, S>), dim3(unsigned(total)), dim3(dl::THREADS),
                     0, s, a);
  return hipGetLastError();
}

// The direct path needs whole 16-byte chunks everywhere: K and every
// K-slow operand's other dimension multiples of 8, 16-byte aligned rows, and
// slices addressable with 32-bit buffer offsets.
inline bool direct_ok(const GemmArgs& a, bool ta, bool tb) {
  if (!a.vec_a || !a.vec_b || a.k % 8 != 0) return false;
  if (ta && a.m % 8 != 0) return false;
  if (!tb && a.n % 8 != 0) return false;
  const int64_t abytes = int64_t(ta ? a.k : a.m) * a.lda * 2;
  const int64_t bbytes = int64_t(tb ? a.n : a.k) * a.ldb * 2;
  return abytes < (int64_t(1) << 31) && bbytes < (int64_t(1) << 31);
}

template <bool X3>
hipError_t dispatch_direct(const GemmArgs& a, bool ta, bool tb, hipStream_t s) {
  constexpr int S = X3 ? 2 : 4;
  if (!ta && !tb) return launch_direct<false, false, X3, S>(a, s);
  if (ta && !tb) return launch_direct<true, false, X3, S>(a, s);
  if (!ta && tb) return launch_direct<false, true, X3, S>(a, s);
  return launch_direct<true, true, X3, S>(a, s);
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
  // The LDS limit is an attribute of the kernel on each device: set it once
  // per instantiation and device (setting it twice is harmless, so a race
  // between host threads costs at most one extra call).
  constexpr int kMaxDevices = 64;
  static std::atomic<bool> attr_set[kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices || !attr_set[dev].load(std::memory_order_acquire)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, D::LDS_BYTES);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < kMaxDevices) attr_set[dev].store(true, std::memory_order_release);
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
  if (direct_ok(a, ta, tb))
    return x3 ? dispatch_direct<true>(a, ta, tb, s) : dispatch_direct<false>(a, ta, tb, s);
  return x3 ? dispatch<CfgBF16, true>(a, ta, tb, s) : dispatch<CfgBF16, false>(a, ta, tb, s);
}

}  // namespace wp
