// MFMA implicit-GEMM kernels for the wide layers (gfx950).
//
// A cached conv is the GEMM  Out[n][m] = sum_kk A[m][kk] * B[kk][n]
// with m the output channel, n a frame of the step's packed frame space
// (frames of all streams back to back, so one tile may span several
// streams), and kk = tap * cin + ci.  Column n of B is gathered from the
// window [cache | new frames] of n's stream: row t * stride + dilation * tap
// for its local output frame t, with LeakyReLU and the operand rounding
// applied on the way into LDS.
//
// A transposed conv with kernel 2r is, per input frame q, the GEMM row block
// m = phi * cout + co over kk = h * cin + ci, where h = 0 reads frame q - 1
// (taps phi + r) and h = 1 reads frame q (taps phi).  Each stream gets one
// extra column q = T that only holds the h = 0 half: it is written as the
// FP32 overlap carry, and column q = 0 of the next buffer starts its
// accumulator from that carry.  Both halves are padded to whole K chunks, so
// every output frame runs the same chain of MFMAs whatever the buffer split.
//
// Precision: FP32 (v_mfma_f32_16x16x4_f32), BF16 RNE (v_mfma_f32_16x16x32_bf16)
// or OCP FP8 e4m3 (v_mfma_scale_f32_16x16x128_f8f6f4, unit block scales) with a
// per-row weight scale and a static activation scale applied in the FP32
// epilogue.  Accumulation, bias, skip, carry and caches are FP32.
//
// Tiling: 256 threads = 4 waves; workgroup tile MT x NT (MT * NT = 4096),
// each wave a 32 x 32 tile = 2 x 2 MFMA 16x16 blocks.  Each K chunk is 128
// bytes of every A row and B column (32 FP32, 64 BF16 or 128 FP8 values); lane
// group g = lane / 16 owns bytes [32g, 32g + 32) of a row, the same slice for A
// and B, so the reduction is over the same K elements for both operands.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "kernels.h"

namespace sc {

namespace {

constexpr int kThreads = 256;
constexpr int kChunkBytes = 128;
constexpr int kRowStride = 144;   // padded LDS row (bytes)

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef int i8v __attribute__((ext_vector_type(8)));
// native 16-byte vector (HIP's uint4 is a union-based class that defeats
// register promotion of arrays of it)
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

template <int PREC> struct Prec;
template <> struct Prec<0> { static constexpr int kEsize = 4; static constexpr int kKc = 32; typedef float Elem; };
template <> struct Prec<1> { static constexpr int kEsize = 2; static constexpr int kKc = 64; typedef uint16_t Elem; };
template <> struct Prec<2> { static constexpr int kEsize = 1; static constexpr int kKc = 128; typedef uint8_t Elem; };

// ---- operand conversion ------------------------------------------------------
__device__ inline uint32_t pack_bf16(float lo, float hi) {
  bf16x2 v = {(__bf16)lo, (__bf16)hi};
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  return u;
}

__device__ inline uint32_t pack_fp8x4(float a, float b, float c, float d) {
  int v = 0;
  v = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(a), sat448(b), v, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(c), sat448(d), v, true);
  return (uint32_t)v;
}

// 32-byte fragment of one lane (its slice of a 128-byte chunk row).
struct Frag {
  u4 lo, hi;
};

template <int PREC>
__device__ inline f4 mfma_chunk(const Frag& a, const Frag& b, f4 acc) {
  if constexpr (PREC == 0) {
    float av[8], bv[8];
    __builtin_memcpy(av, &a, 32);
    __builtin_memcpy(bv, &b, 32);
#pragma unroll
    for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
  } else if constexpr (PREC == 1) {
    bf16x8 a0, a1, b0, b1;
    __builtin_memcpy(&a0, &a.lo, 16);
    __builtin_memcpy(&a1, &a.hi, 16);
    __builtin_memcpy(&b0, &b.lo, 16);
    __builtin_memcpy(&b1, &b.hi, 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
  } else {
    i8v av, bv;
    __builtin_memcpy(&av, &a, 32);
    __builtin_memcpy(&bv, &b, 32);
    // formats 0/0 = FP8 e4m3 for both operands; E8M0 block scales 127 = 1.0
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, 127, 0, 127);
  }
  return acc;
}

// Per-column context of a tile, staged in LDS once per tile.
struct ColInfo {
  const float* cache;   // conv: current cache copy of the column's stream (raw FP32 [L][cin])
  const unsigned char* tcache;   // conv: current twin cache copy (operand type [L][cin])
  int32_t ei;           // entry (stream) index; -1 for a padding column
  int32_t t;            // conv: local output frame; convt: q (== Tin for a carry column)
  int32_t in_start;     // first packed input frame of the stream
  int32_t Tin;          // input frames of the stream
  int32_t keep_lo, keep_hi;   // local output frames outside [keep_lo, keep_hi) are zeroed (masks)
  int32_t parity;       // the stream's current state copy (the other one is written)
};

template <bool CONVT>
__device__ inline ColInfo make_col(const LayerArgs& a, int32_t n, int32_t n_cols) {
  ColInfo c;
  c.cache = nullptr;
  c.tcache = nullptr;
  c.ei = -1;
  c.t = 0;
  c.in_start = 0;
  c.Tin = 0;
  c.keep_lo = 0;
  c.keep_hi = 0;
  c.parity = 0;
  if (n >= n_cols) return c;
  int ei;
  if (CONVT) ei = n < step_in(a) ? entry_of_in(a, n) : n - (int32_t)step_in(a);
  else ei = entry_of_out(a, n);
  const Entry e = load_entry(a.ents + ei);
  c.ei = ei;
  c.in_start = in_frames(a, e.off);
  c.Tin = in_frames(a, e.T);
  c.cache = e.state + a.state_off + (int64_t)e.parity * a.state_len;   // conv cache / convt carry copy
  c.parity = e.parity;
  keep_range(e, a.delay, a.out_num, a.out_den, &c.keep_lo, &c.keep_hi);
  if (CONVT) {
    c.t = n < step_in(a) ? n - c.in_start : c.Tin;
  } else {
    c.t = n - out_frames(a, e.off);
    c.tcache = reinterpret_cast<const unsigned char*>(e.state + a.tstate_off + (int64_t)e.parity * a.tstate_len);
  }
  return c;
}

template <int PREC>
__device__ inline void store4(unsigned char* dst, float v0, float v1, float v2, float v3) {
  if constexpr (PREC == 0) {
    *reinterpret_cast<f4*>(dst) = f4{v0, v1, v2, v3};
  } else if constexpr (PREC == 1) {
    uint2 u;
    u.x = pack_bf16(v0, v1);
    u.y = pack_bf16(v2, v3);
    *reinterpret_cast<uint2*>(dst) = u;
  } else {
    *reinterpret_cast<uint32_t*>(dst) = pack_fp8x4(v0, v1, v2, v3);
  }
}

// Writes the operand twin of 4 consecutive output elements (element index o)
// in the consumer's operand type (an FP32 layer may feed a reduced-precision one).
template <int PREC>
__device__ inline void store_twin4(const LayerArgs& a, int64_t o, f4 v) {
  if (a.twin_pre) {
    v.x = lrelu(v.x);
    v.y = lrelu(v.y);
    v.z = lrelu(v.z);
    v.w = lrelu(v.w);
  }
  const float q = a.twin_qs;
  unsigned char* dst = static_cast<unsigned char*>(a.out_twin);
  if (a.twin_prec == PREC) store4<PREC>(dst + o * Prec<PREC>::kEsize, v.x * q, v.y * q, v.z * q, v.w * q);
  else if (a.twin_prec == 0) store4<0>(dst + o * 4, v.x * q, v.y * q, v.z * q, v.w * q);
  else if (a.twin_prec == 1) store4<1>(dst + o * 2, v.x * q, v.y * q, v.z * q, v.w * q);
  else store4<2>(dst + o, v.x * q, v.y * q, v.z * q, v.w * q);
}

// A 2-chunk register pipeline; kernels reading operand twins ask for 4 waves
// per SIMD (3 for FP8), measured faster than 4 chunks in flight at 3 waves;
// the others keep the default register budget (they would spill).
template <int PREC, int MT, int NT, bool CONVT, bool INTWIN>
__global__ void __launch_bounds__(kThreads, INTWIN ? (PREC == 2 ? 3 : 4) : 1) gemm_kernel(LayerArgs a, int32_t n_cols, int n_mt, int n_nt,
                                                        int Kpad, int Kreal, int half_pad, int Mreal,
                                                        int extra_blocks, FastDiv fd_per_ent) {
  constexpr int KC = Prec<PREC>::kKc;
  constexpr int ES = Prec<PREC>::kEsize;
  constexpr int WM = MT / 32;                   // waves along M
  static_assert(WM * (NT / 32) == 4, "4 waves of 32x32");
  constexpr int A_PIECES = MT * 8 / kThreads;
  static_assert(A_PIECES == 1 || A_PIECES == 2, "MT of 32 or 64");

  __shared__ __attribute__((aligned(16))) unsigned char lds_a[2][MT * kRowStride];
  __shared__ __attribute__((aligned(16))) unsigned char lds_b[2][NT * kRowStride];
  __shared__ ColInfo cols[NT];

  const int tid = threadIdx.x;
  const int32_t n_tiles = n_mt * n_nt;   // tiles of the grid (sized for the largest step)
  int32_t bid = blockIdx.x;
  // ---- conv cache update blocks (after the GEMM tiles): 4 channels per item ----
  if (!CONVT && bid >= n_tiles) {
    const int32_t per_ent = a.L * a.cin / 4;   // cin is a multiple of 4
    const int32_t total = step_ents(a) * per_ent;
    for (int32_t j = (bid - n_tiles) * kThreads + tid; j < total; j += extra_blocks * kThreads) {
      const int ei = (int)fdiv(fd_per_ent, (uint32_t)j);
      const int32_t rem = (j - ei * per_ent) * 4;
      const int32_t i = (int32_t)fdiv(a.fd_cin, (uint32_t)rem);
      const int ci = rem - i * a.cin;
      const Entry e = load_entry(a.ents + ei);
      const int32_t Tin = in_frames(a, e.T);
      const int32_t row = Tin + i;
      const int64_t src_in = ((int64_t)in_frames(a, e.off) + row - a.L) * a.cin + ci;
      const float* src = row < a.L ? e.state + a.state_off + (int64_t)e.parity * a.state_len + (int64_t)row * a.cin + ci
                                   : a.in_buf + src_in;
      f4 v;
      if (PREC == 0 && MT == 64 && !INTWIN && a.user_in && row >= a.L) {
        // the caller's channel-major buffer: channels ci .. ci + 3 of input frame row - L
        const float* u = e.in + (int64_t)ci * e.T + (row - a.L);
        v = f4{gload<float>(u), gload<float>(u + e.T), gload<float>(u + 2 * (int64_t)e.T),
               gload<float>(u + 3 * (int64_t)e.T)};
      } else {
        v = gload<f4>(src);
      }
      gstore<f4>(e.state + a.state_off + (int64_t)(1 - e.parity) * a.state_len + (int64_t)i * a.cin + ci, v);
      if (INTWIN) {
        // 4 operand elements: 16, 8 or 4 bytes
        typedef typename Prec<PREC>::Elem T;
        const T* tsrc = row < a.L
            ? reinterpret_cast<const T*>(e.state + a.tstate_off + (int64_t)e.parity * a.tstate_len) + (int64_t)row * a.cin + ci
            : static_cast<const T*>(a.in_twin) + src_in;
        T* tdst = reinterpret_cast<T*>(e.state + a.tstate_off + (int64_t)(1 - e.parity) * a.tstate_len) +
                  (int64_t)i * a.cin + ci;
        if constexpr (sizeof(T) == 4) gstore<u4>(tdst, gload<u4>(tsrc));
        else if constexpr (sizeof(T) == 2) gstore<uint64_t>(tdst, gload<uint64_t>(tsrc));
        else gstore<uint32_t>(tdst, gload<uint32_t>(tsrc));
      }
    }
    return;
  }
  // the grid may be sized for a larger step than this one (captured launches):
  // the step's own tiles are the first ones
  n_cols = CONVT ? step_in(a) + step_ents(a) : step_out(a);
  const int32_t step_tiles = n_mt * ((n_cols + NT - 1) / NT);
  if (bid >= step_tiles) return;
  // XCD-aware order: consecutive blocks go round-robin to the 8 XCDs; remap so
  // that the M tiles of one column tile (which share B) run on one XCD's L2
  {
    const int32_t full = step_tiles / 8 * 8;
    if (bid < full) bid = (bid % 8) * (full / 8) + bid / 8;
  }
  const int mt = (int)((uint32_t)bid % (uint32_t)n_mt);
  const int32_t nt = (int32_t)((uint32_t)bid / (uint32_t)n_mt);
  const int m0 = mt * MT;
  const int32_t n0 = nt * NT;

  const unsigned char* Wb = static_cast<const unsigned char*>(a.W);
  const int row_bytes = Kpad * ES;
  const int n_chunks = Kpad / KC;
  const bool pre = a.pre_act != 0;
  const float qs = (PREC == 2) ? 1.0f / a.act_scale : 1.0f;

  // Register pipeline: chunk c + STAGES is in flight while chunk c is
  // multiplied, so a chunk's memory latency overlaps STAGES chunks of work.
  constexpr int STAGES = 2;
  static_assert(STAGES == 2 || STAGES == 4, "stages are written out for 2 or 4");
  constexpr int EPP = INTWIN ? 16 / ES : 4;             // elements per B piece
  constexpr int PPCOL = KC / EPP;                       // pieces per column per chunk
  constexpr int B_PIECES = NT * PPCOL / kThreads;       // pieces per thread per chunk
  static_assert(B_PIECES >= 1 && NT * PPCOL % kThreads == 0 && kThreads % PPCOL == 0, "piece mapping");
  const int my_pp = tid % PPCOL;                        // piece index within a column chunk (fixed)
  const int my_col0 = tid / PPCOL;                      // first column; then + kThreads / PPCOL
  u4 ar0[STAGES], ar1[STAGES];                       // A pieces (16 B) per stage
  u4 tb[STAGES][INTWIN ? B_PIECES : 1];              // B twin pieces
  f4 rb[STAGES][INTWIN ? 1 : B_PIECES];                 // B raw FP32 pieces

  // ---- pipeline stage operations (macros: the stage registers must stay
  // in VGPRs, which lambdas over arrays defeat) ----
#define SC_LOAD_A(C, ST)                                                                                     \
  {                                                                                                          \
    const int r_ = tid >> 3, seg_ = tid & 7;                                                                 \
    ar0[ST] = *reinterpret_cast<const u4*>(Wb + (int64_t)(m0 + r_) * row_bytes + (C) * kChunkBytes + seg_ * 16); \
    if constexpr (A_PIECES == 2)                                                                             \
      ar1[ST] = *reinterpret_cast<const u4*>(Wb + (int64_t)(m0 + r_ + 32) * row_bytes + (C) * kChunkBytes +      \
                                                seg_ * 16);                                                  \
  }
#define SC_LOAD_B(C, ST)                                                                                     \
  {                                                                                                          \
    const int drow_ = a.dil * k_tap;                                   /* conv: tap offset in rows */        \
    const int64_t koff_ = (int64_t)drow_ * a.cin + k_ci;               /* conv: elements past (t, 0) */      \
    _Pragma("unroll") for (int p_ = 0; p_ < B_PIECES; ++p_) {                                                \
      bool live_;                                                                                            \
      int64_t off_;                                                                                          \
      const unsigned char* base_ = in_base;                                                                  \
      if (CONVT) {                                                                                           \
        const int kk_ = (C) * KC + my_pp * EPP;                                                              \
        const int h_ = kk_ >= half_pad;                                                                      \
        const int ci_ = kk_ - h_ * half_pad;                                                                 \
        const int row_ = pc_t[p_] - 1 + h_;                                                                  \
        live_ = pc_ok[p_] && ci_ < a.cin && row_ >= 0 && row_ < pc_lim[p_];                                   \
        off_ = pc_in[p_] + (int64_t)row_ * a.cin + ci_;                                                      \
      } else {                                                                                               \
        /* window row t + dil tap: the cache copy below L, the input above */                                \
        live_ = pc_ok[p_] && (C) * KC + my_pp * EPP < Kreal;                                                 \
        base_ = pc_t[p_] + drow_ < a.L ? pc_cache[p_] : pc_inb[p_];                                          \
        off_ = koff_;                                                                                        \
      }                                                                                                      \
      if constexpr (INTWIN) {                                                                                \
        tb[ST][p_] = live_ ? gload<u4>(base_ + off_ * ES) : u4{0u, 0u, 0u, 0u};                         \
      } else if (PREC == 0 && MT == 64 && !CONVT && a.user_in && pc_t[p_] + drow_ >= a.L) {                  \
        /* the caller's channel-major buffer: channels k_ci .. + 3 of the row, T_e apart */                  \
        const int64_t ut_ = pc_ut[PREC == 0 && MT == 64 && !INTWIN && !CONVT ? p_ : 0];                                 \
        const float* u_ = reinterpret_cast<const float*>(pc_inb[p_]) + drow_ + (int64_t)k_ci * ut_;           \
        rb[ST][p_] = live_ ? f4{gload<float>(u_), gload<float>(u_ + ut_), gload<float>(u_ + 2 * ut_),         \
                                gload<float>(u_ + 3 * ut_)}                                                  \
                           : f4{0.f, 0.f, 0.f, 0.f};                                                         \
      } else {                                                                                               \
        rb[ST][p_] = live_ ? gload<f4>(base_ + off_ * 4) : f4{0.f, 0.f, 0.f, 0.f};                       \
      }                                                                                                      \
    }                                                                                                        \
    if (!CONVT) {                                                                                            \
      k_ci += KC;                                                                                            \
      while (k_ci >= a.cin) {                                                                                \
        k_ci -= a.cin;                                                                                       \
        ++k_tap;                                                                                             \
      }                                                                                                      \
    }                                                                                                        \
  }
#define SC_STORE(BUF, ST)                                                                                    \
  {                                                                                                          \
    const int r_ = tid >> 3, seg_ = tid & 7;                                                                 \
    *reinterpret_cast<u4*>(&lds_a[BUF][r_ * kRowStride + seg_ * 16]) = ar0[ST];                           \
    if constexpr (A_PIECES == 2) *reinterpret_cast<u4*>(&lds_a[BUF][(r_ + 32) * kRowStride + seg_ * 16]) = ar1[ST]; \
    _Pragma("unroll") for (int p_ = 0; p_ < B_PIECES; ++p_) {                                                \
      const int col_ = my_col0 + p_ * (kThreads / PPCOL);                                                    \
      unsigned char* dst_ = &lds_b[BUF][col_ * kRowStride + my_pp * EPP * ES];                               \
      if constexpr (INTWIN) {                                                                                \
        *reinterpret_cast<u4*>(dst_) = tb[ST][p_];                                                        \
      } else {                                                                                               \
        f4 v_ = rb[ST][p_];                                                                                  \
        if (pre) {                                                                                           \
          v_.x = lrelu(v_.x);                                                                                \
          v_.y = lrelu(v_.y);                                                                                \
          v_.z = lrelu(v_.z);                                                                                \
          v_.w = lrelu(v_.w);                                                                                \
        }                                                                                                    \
        store4<PREC>(dst_, v_.x * qs, v_.y * qs, v_.z * qs, v_.w * qs);                                      \
      }                                                                                                      \
    }                                                                                                        \
  }

  // the weight pieces do not depend on the columns: start them first
  // (stages written out: the stage registers need compile-time indices)
  SC_LOAD_A(0, 0)
  if (1 < n_chunks) SC_LOAD_A(1, 1)
  if constexpr (STAGES > 2) {
    if (2 < n_chunks) SC_LOAD_A(2, 2)
    if (3 < n_chunks) SC_LOAD_A(3, 3)
  }

  if (tid < NT) cols[tid] = make_col<CONVT>(a, n0 + tid, n_cols);
  __syncthreads();

  // the columns of this thread's B pieces are the same for every K chunk:
  // their gather context lives in registers (no LDS reads in the K loop)
  const unsigned char* in_base = INTWIN ? static_cast<const unsigned char*>(a.in_twin)
                                        : reinterpret_cast<const unsigned char*>(a.in_buf);
  constexpr int ES_B = INTWIN ? ES : 4;      // bytes per B source element
  // conv: pc_cache / pc_inb address window row t of the column (element 0) in
  // the cache copy and in the input; a chunk adds the thread's tap and channel
  const unsigned char* pc_cache[B_PIECES];
  const unsigned char* pc_inb[B_PIECES];
  int64_t pc_in[B_PIECES];                   // convt: input element offset of the stream's frame 0
  int32_t pc_t[B_PIECES];                    // conv: window row of tap 0 (t * stride); convt: q
  int32_t pc_lim[B_PIECES];                  // convt: input frames of the stream
  int32_t pc_ut[PREC == 0 && MT == 64 && !INTWIN && !CONVT ? B_PIECES : 1];   // direct model input: channel stride (the stream's T)
  bool pc_ok[B_PIECES];                      // not a padding column
#pragma unroll
  for (int p = 0; p < B_PIECES; ++p) {
    const ColInfo& cc = cols[my_col0 + p * (kThreads / PPCOL)];
    pc_ok[p] = cc.ei >= 0;
    pc_t[p] = CONVT ? cc.t : cc.t * a.stride;   // conv: the window row of tap 0
    pc_lim[p] = cc.Tin;
    pc_in[p] = (int64_t)cc.in_start * a.cin;
    const int64_t trow = (int64_t)pc_t[p] * a.cin;
    pc_cache[p] = (INTWIN ? cc.tcache : reinterpret_cast<const unsigned char*>(cc.cache)) + trow * ES_B;
    pc_inb[p] = in_base + (((int64_t)cc.in_start - a.L) * a.cin + trow) * ES_B;
    if (PREC == 0 && MT == 64 && !INTWIN && !CONVT) pc_ut[p] = 0;
    if (PREC == 0 && MT == 64 && !INTWIN && !CONVT && a.user_in) {
      // input row r of the column's stream is element (ci, r) of its buffer at in + ci * T + r
      const Entry e = load_entry(a.ents + max(cc.ei, 0));
      pc_inb[p] = reinterpret_cast<const unsigned char*>(e.in + ((int64_t)pc_t[p] - a.L));
      pc_ut[p] = e.T;
    }
  }

  // K position of this thread's B piece, advanced chunk by chunk without
  // division (chunks are gathered in increasing order)
  int k_tap = 0, k_ci = 0;
  if (!CONVT) {
    const int kk0 = my_pp * EPP;
    k_tap = (int)fdiv(a.fd_cin, (uint32_t)kk0);
    k_ci = kk0 - k_tap * a.cin;
  }
  SC_LOAD_B(0, 0)
  if (1 < n_chunks) SC_LOAD_B(1, 1)
  if constexpr (STAGES > 2) {
    if (2 < n_chunks) SC_LOAD_B(2, 2)
    if (3 < n_chunks) SC_LOAD_B(3, 3)
  }

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lg = lane >> 4;

  // accumulators; a transposed conv's column q = 0 starts from the carry
  f4 acc[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const ColInfo& cj = cols[wn * 32 + j * 16 + lr];
    const bool from_carry = CONVT && cj.ei >= 0 && cj.t == 0 && cj.Tin > 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // the lane's rows of this 16-row block: m .. m + 3
      const int m = m0 + wm * 32 + i * 16 + lg * 4;
      f4 cv = {0.f, 0.f, 0.f, 0.f};
      if (from_carry && m < Mreal) cv = gload<f4>(cj.cache + m);
      acc[i][j] = cv;
    }
  }

#define SC_STAGE(ST)                                                                                         \
  {                                                                                                          \
    const int c = c0 + (ST);                                                                                 \
    if (c < n_chunks) {                                                                                      \
      const int buf = c & 1;                                                                                 \
      SC_STORE(buf, ST)                                                                                      \
      __syncthreads();                                                                                       \
      if (c + STAGES < n_chunks) {                                                                           \
        SC_LOAD_A(c + STAGES, ST)                                                                            \
        SC_LOAD_B(c + STAGES, ST)                                                                            \
      }                                                                                                      \
      Frag fa[2], fb[2];                                                                                     \
      _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                                        \
        const unsigned char* p = &lds_a[buf][(wm * 32 + i * 16 + lr) * kRowStride + lg * 32];               \
        fa[i].lo = *reinterpret_cast<const u4*>(p);                                                       \
        fa[i].hi = *reinterpret_cast<const u4*>(p + 16);                                                  \
      }                                                                                                      \
      _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                                        \
        const unsigned char* p = &lds_b[buf][(wn * 32 + j * 16 + lr) * kRowStride + lg * 32];               \
        fb[j].lo = *reinterpret_cast<const u4*>(p);                                                       \
        fb[j].hi = *reinterpret_cast<const u4*>(p + 16);                                                  \
      }                                                                                                      \
      _Pragma("unroll") for (int i = 0; i < 2; ++i)                                                          \
        _Pragma("unroll") for (int j = 0; j < 2; ++j) acc[i][j] = mfma_chunk<PREC>(fa[i], fb[j], acc[i][j]); \
    }                                                                                                        \
  }
  // epilogue operands (bias, FP8 row scales, residual skip rows) are fetched
  // now so that their latency hides behind the K loop
  f4 ep_bias[2], ep_ws[2], ep_skip[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + wm * 32 + i * 16 + lg * 4;
    const bool ok = m < Mreal;
    const int co = CONVT ? m - (int)fdiv(a.fd_cout, (uint32_t)m) * a.cout : m;
    ep_bias[i] = ok ? *reinterpret_cast<const f4*>(a.B + co) : f4{0.f, 0.f, 0.f, 0.f};
    ep_ws[i] = (PREC == 2 && ok) ? *reinterpret_cast<const f4*>(a.wscale + m) : f4{1.f, 1.f, 1.f, 1.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      ep_skip[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      if (!CONVT && ok && a.residual) {
        const ColInfo& c = cols[wn * 32 + j * 16 + lr];
        if (c.ei >= 0) {
          const int row = c.t + a.skip_off;
          const float* sp = row < a.L ? c.cache + (int64_t)row * a.cin
                                      : a.in_buf + ((int64_t)c.in_start + row - a.L) * a.cin;
          ep_skip[i][j] = gload<f4>(sp + m);
        }
      }
    }
  }

  for (int c0 = 0; c0 < n_chunks; c0 += STAGES) {
    SC_STAGE(0)
    SC_STAGE(1)
    if constexpr (STAGES > 2) {
      SC_STAGE(2)
      SC_STAGE(3)
    }
  }
#undef SC_STAGE

#undef SC_LOAD_A
#undef SC_LOAD_B
#undef SC_STORE

  // ---- epilogue: lane holds rows m..m+3 of column n for each (i, j) ----
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const ColInfo& c = cols[wn * 32 + j * 16 + lr];
    if (c.ei < 0) continue;
    const int32_t n = n0 + wn * 32 + j * 16 + lr;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + wm * 32 + i * 16 + lg * 4;
      if (m >= Mreal) continue;
      f4 v = acc[i][j];
      if (PREC == 2) v = v * (ep_ws[i] * a.act_scale);
      if (CONVT) {
        if (c.t >= c.Tin) {
          // carry column: FP32 partial sums of the next buffer's first frame,
          // kept in accumulator units (before the FP8 dequantization)
          float* carry_out = const_cast<float*>(c.cache) + (int64_t)(1 - 2 * c.parity) * a.state_len;
          gstore<f4>(carry_out + m, acc[i][j]);
          continue;
        }
        const int phi = (int)fdiv(a.fd_cout, (uint32_t)m);
        v = v + ep_bias[i];
        const int32_t t = c.t * a.stride + phi;
        if (t < c.keep_lo || t >= c.keep_hi) v = f4{0.f, 0.f, 0.f, 0.f};
        const int64_t o = ((int64_t)c.in_start * a.stride + (int64_t)c.t * a.stride) * a.cout + m;
        if (!a.twin_only) gstore<f4>(a.out_buf + o, v);
        if (a.out_twin) store_twin4<PREC>(a, o, v);
      } else {
        v = v + ep_bias[i];
        if (a.residual) v = v + ep_skip[i][j];
        if (c.t < c.keep_lo || c.t >= c.keep_hi) v = f4{0.f, 0.f, 0.f, 0.f};
        if (!a.twin_only) gstore<f4>(a.out_buf + (int64_t)n * a.cout + m, v);
        if (a.out_twin) store_twin4<PREC>(a, (int64_t)n * a.cout + m, v);
      }
    }
  }
}

// ---- host side -------------------------------------------------------------------
int esize(int prec) { return prec == 0 ? 4 : (prec == 1 ? 2 : 1); }
int kchunk(int prec) { return prec == 0 ? 32 : (prec == 1 ? 64 : 128); }
int round_up(int x, int m) { return (x + m - 1) / m * m; }

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// OCP FP8 E4M3FN, round to nearest even, saturating to +-448 (finite input).
uint8_t fp8_e4m3_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint8_t sign = (u >> 31) ? 0x80 : 0;
  float a = std::fabs(f);
  if (!(a > 0.f)) return sign;
  if (a >= 448.f) return sign | 0x7E;
  int e;
  std::frexp(a, &e);              // a = m * 2^e, m in [0.5, 1)
  int exp = e - 1;                // a = 1.f * 2^exp
  if (exp < -6) exp = -6;         // subnormal range shares the minimum exponent
  const float q = std::ldexp(a, 3 - exp);   // value in units of the ulp (2^(exp-3))
  float r = std::nearbyint(q);             // ties to even under the default rounding mode
  int mant = (int)r;
  if (mant >= 16) { exp += 1; mant >>= 1; }  // carried into the next binade
  if (exp > 8 || (exp == 8 && mant > 14)) return sign | 0x7E;
  if (mant < 8) return sign | (uint8_t)mant;                      // subnormal (exp == -6)
  return sign | (uint8_t)(((exp + 7) << 3) | (mant - 8));
}

// Packs rows of FP32 values (row m of length Kreal values, mapped into a padded
// row by `kpos`) into the operand type; FP8 gets a per-row scale.
template <class RowFn, class PosFn>
void pack_rows(int M, int Mpad, int Kpad, int prec, RowFn value, PosFn kpos, int Kreal, std::vector<uint8_t>& out,
               std::vector<float>& wscale) {
  const int es = esize(prec);
  out.assign((size_t)Mpad * Kpad * es, 0);
  if (prec == 2) wscale.assign((size_t)Mpad, 1.0f);
  for (int m = 0; m < M; ++m) {
    float s = 1.0f;
    if (prec == 2) {
      float amax = 0.f;
      for (int k = 0; k < Kreal; ++k) amax = std::max(amax, std::fabs(value(m, k)));
      s = amax > 0.f ? amax / 448.f : 1.0f;
      wscale[m] = s;
    }
    for (int k = 0; k < Kreal; ++k) {
      const float w = value(m, k);
      uint8_t* dst = &out[((size_t)m * Kpad + kpos(k)) * es];
      if (prec == 0) {
        std::memcpy(dst, &w, 4);
      } else if (prec == 1) {
        const uint16_t h = bf16_rne(w);
        std::memcpy(dst, &h, 2);
      } else {
        *dst = fp8_e4m3_rne(w / s);
      }
    }
  }
}

// Tile shape per GEMM M (output rows).  A conv whose M is an odd multiple of
// 32 (96 channels) takes 32 x 128 tiles, which leave no padding rows: measured
// 10% faster than 64 x 64 tiles on the 96-channel convs; the transposed conv
// of that M measured faster on 64 x 64.
void tile_for(int M, bool convt, int& MT, int& NT) {
  if (M <= 32 || (!convt && M % 64 == 32)) { MT = 32; NT = 128; }
  else { MT = 64; NT = 64; }
}

template <int PREC, int MT, int NT, bool CONVT, bool INTWIN>
hipError_t launch_t(const LayerArgs& a, int64_t n_cols, int Kpad, int Kreal, int half_pad, int M,
                    hipStream_t s) {
  const int n_mt = (M + MT - 1) / MT;
  const int64_t n_nt = (n_cols + NT - 1) / NT;
  int extra = 0;
  if (!CONVT) {
    const int64_t items = (int64_t)a.n_ent * a.L * a.cin / 4;   // 4 channels per item
    extra = (int)std::min<int64_t>((items + kThreads - 1) / kThreads, 1024);
  }
  const int64_t grid = (int64_t)n_mt * n_nt + extra;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_kernel<PREC, MT, NT, CONVT, INTWIN>), dim3((unsigned)grid), dim3(kThreads), 0, s, a,
                     (int32_t)n_cols, n_mt, (int)n_nt, Kpad, Kreal, half_pad, M, extra,
                     make_fastdiv((uint32_t)std::max(a.L * a.cin / 4, 1)));
  return hipGetLastError();
}

template <bool CONVT>
hipError_t dispatch(const LayerArgs& a, int prec, int64_t n_cols, int Kpad, int Kreal, int half_pad, int M,
                    hipStream_t s) {
  int MT, NT;
  tile_for(M, CONVT, MT, NT);
#define SC_CASE(P, A, B)                                                                                   \
  if (prec == P && MT == A && NT == B) {                                                                   \
    if (a.in_twin) return launch_t<P, A, B, CONVT, true>(a, n_cols, Kpad, Kreal, half_pad, M, s);         \
    return launch_t<P, A, B, CONVT, false>(a, n_cols, Kpad, Kreal, half_pad, M, s);                       \
  }
  SC_CASE(0, 32, 128) SC_CASE(0, 64, 64)
  SC_CASE(1, 32, 128) SC_CASE(1, 64, 64)
  SC_CASE(2, 32, 128) SC_CASE(2, 64, 64)
#undef SC_CASE
  return hipErrorInvalidValue;
}

}  // namespace

bool conv_mfma_supported(int cin, int cout, int k, int stride, int prec) {
  (void)k;
  // 16-byte operand pieces never straddle two taps: cin * element size % 16 == 0.
  // Stride-1 convs narrower than 32 input channels stay on the wavefront
  // kernels (measured faster there, and the decoder's 16-channel input conv
  // must not round its input); strided ones have no fast wavefront form.
  const int es = esize(prec);
  return stride >= 1 && (cin * es) % 16 == 0 && cin % 8 == 0 && cout % 16 == 0 &&
         cin >= (stride > 1 ? 16 : 32) && cout >= 16 && prec >= 0 && prec <= 2;
}

bool conv_mfma_fp32_input_supported(int cin, int cout, int k, int stride) {
  (void)k;
  // FP32 operands: 16-byte pieces of 4 channels never straddle two taps
  return stride == 1 && cin % 4 == 0 && cin >= 4 && cout % 16 == 0 && cout >= 32;
}

bool convt_mfma_supported(int cin, int cout, int r, int prec) {
  const int es = esize(prec);
  return (cin * es) % 16 == 0 && cin % 8 == 0 && cout % 4 == 0 && cin >= 32 && r * cout >= 32 &&
         (r * cout) % 16 == 0 && prec >= 0 && prec <= 2;
}

void pack_conv_mfma(const float* w, int cout, int cin, int k, int prec, std::vector<uint8_t>& out,
                    std::vector<float>& wscale) {
  int MT, NT;
  tile_for(cout, false, MT, NT);
  const int Kreal = k * cin;
  const int Kpad = round_up(Kreal, kchunk(prec));
  const int Mpad = round_up(cout, MT);
  // row m, column kk = tap * cin + ci  <-  W[m][ci][tap]
  pack_rows(cout, Mpad, Kpad, prec,
            [&](int m, int kk) { const int tap = kk / cin, ci = kk % cin; return w[((size_t)m * cin + ci) * k + tap]; },
            [](int kk) { return kk; }, Kreal, out, wscale);
}

void pack_convt_mfma(const float* w, int cin, int cout, int r, int prec, std::vector<uint8_t>& out,
                     std::vector<float>& wscale) {
  const int M = r * cout;
  int MT, NT;
  tile_for(M, true, MT, NT);
  const int half = round_up(cin, kchunk(prec));
  const int Kpad = 2 * half;
  const int Mpad = round_up(M, MT);
  // row m = phi * cout + co; column kk = h * cin + ci: h = 0 -> tap phi + r, h = 1 -> tap phi
  pack_rows(M, Mpad, Kpad, prec,
            [&](int m, int kk) {
              const int phi = m / cout, co = m % cout;
              const int h = kk / cin, ci = kk % cin;
              const int tap = h == 0 ? phi + r : phi;
              return w[((size_t)ci * cout + co) * (2 * r) + tap];
            },
            [&](int kk) { return (kk / cin) * half + kk % cin; }, 2 * cin, out, wscale);
}

hipError_t launch_conv_mfma(const LayerArgs& a, int prec, hipStream_t s) {
  const int Kreal = a.k * a.cin;
  const int Kpad = round_up(Kreal, kchunk(prec));
  return dispatch<false>(a, prec, a.n_out, Kpad, Kreal, 0, a.cout, s);
}

hipError_t launch_convt_mfma(const LayerArgs& a, int prec, hipStream_t s) {
  const int half = round_up(a.cin, kchunk(prec));
  return dispatch<true>(a, prec, a.n_in + a.n_ent, 2 * half, 2 * a.cin, half, a.stride * a.cout, s);
}

}  // namespace sc
