// LDS-window MFMA kernel for cached stride-1 convs with narrow inputs (gfx950).
//
// Cached padding (Sec. 2.2): output frame t of a stream reads rows
// t + dil * tap of that stream's window [cache (L frames) | new frames].  A
// workgroup computes output rows [m0, m0 + MT) for F consecutive frames of the
// step's packed frame space.  Those frames may belong to a few streams; for
// each of them the workgroup copies, once, the window rows its columns read
// (the columns' own rows plus the L rows behind the first of them) into LDS as
// raw FP32, back to back.  Column c then finds the row of tap `tap` at
// colbase[c] + dil * tap, whatever stream it belongs to; the residual skip is
// the row colbase[c] + skip_off of the same staged rows.  LeakyReLU and the
// operand rounding (BF16 RNE, or FP8 e4m3 with the layer's static activation
// scale) are applied on the way from LDS into the MFMA registers.
//
// Compared with the gather kernel this reads every input element from HBM
// once per tile (plus the L-row halo), keeps all per-element address work out
// of the K loop, and needs no pre-rounded operand copy from the producer.
//
// The reduction order over K is that of the gather kernel (same packed
// weights, same 128-byte chunks, same MFMA instructions), so both kernels
// produce the same bits for the same layer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace sc {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxStreams = 8;     // streams one tile may touch (the host guarantees it)
constexpr int kStageBatch = 6;     // 16-byte staging loads in flight per thread (fits 5 waves per SIMD)

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));

template <int PREC> struct WPrec;
template <> struct WPrec<0> { static constexpr int kEsize = 4; static constexpr int kKc = 32; };
template <> struct WPrec<1> { static constexpr int kEsize = 2; static constexpr int kKc = 64; };
template <> struct WPrec<2> { static constexpr int kEsize = 1; static constexpr int kKc = 128; };

__device__ inline uint32_t wpack_bf16(float lo, float hi) {
  bf16x2 v = {(__bf16)lo, (__bf16)hi};
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  return u;
}

__device__ inline uint32_t wpack_fp8x4(float a, float b, float c, float d) {
  int v = 0;
  v = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(a), sat448(b), v, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(c), sat448(d), v, true);
  return (uint32_t)v;
}

__device__ inline float act(float v, bool pre) { return pre ? lrelu(v) : v; }

__device__ inline int w_esize_dev(int prec) { return prec == 0 ? 4 : (prec == 1 ? 2 : 1); }

// 16 bytes of operand (4 FP32, 8 BF16 or 16 FP8 values) from FP32 values in LDS
// starting at p, with the pre-activation and the FP8 activation scale.
template <int PREC>
__device__ inline u4 operand16(const float* p, bool pre, float qs) {
  u4 r;
  if constexpr (PREC == 0) {
    const f4 v = *reinterpret_cast<const f4*>(p);
    r[0] = __float_as_uint(act(v.x, pre));
    r[1] = __float_as_uint(act(v.y, pre));
    r[2] = __float_as_uint(act(v.z, pre));
    r[3] = __float_as_uint(act(v.w, pre));
  } else if constexpr (PREC == 1) {
    const f4 v0 = *reinterpret_cast<const f4*>(p);
    const f4 v1 = *reinterpret_cast<const f4*>(p + 4);
    r[0] = wpack_bf16(act(v0.x, pre), act(v0.y, pre));
    r[1] = wpack_bf16(act(v0.z, pre), act(v0.w, pre));
    r[2] = wpack_bf16(act(v1.x, pre), act(v1.y, pre));
    r[3] = wpack_bf16(act(v1.z, pre), act(v1.w, pre));
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f4 v = *reinterpret_cast<const f4*>(p + 4 * q);
      r[q] = wpack_fp8x4(act(v.x, pre) * qs, act(v.y, pre) * qs, act(v.z, pre) * qs, act(v.w, pre) * qs);
    }
  }
  return r;
}

// Four FP32 values in operand form (pre-activation, FP8 activation scale) at dst.
template <int PREC>
__device__ inline void store_operand(unsigned char* dst, f4 v, bool pre, float qs) {
  if constexpr (PREC == 0) {
    *reinterpret_cast<f4*>(dst) = f4{act(v.x, pre), act(v.y, pre), act(v.z, pre), act(v.w, pre)};
  } else if constexpr (PREC == 1) {
    uint2 w;
    w.x = wpack_bf16(act(v.x, pre), act(v.y, pre));
    w.y = wpack_bf16(act(v.z, pre), act(v.w, pre));
    *reinterpret_cast<uint2*>(dst) = w;
  } else {
    *reinterpret_cast<uint32_t*>(dst) =
        wpack_fp8x4(act(v.x, pre) * qs, act(v.y, pre) * qs, act(v.z, pre) * qs, act(v.w, pre) * qs);
  }
}

// The operand copy of output elements o .. o + 3 for the layer's reader, in its type.
__device__ inline void store_twin(const LayerArgs& a, int64_t o, f4 v) {
  f4 w = v;
  if (a.twin_pre) {
    w.x = lrelu(w.x);
    w.y = lrelu(w.y);
    w.z = lrelu(w.z);
    w.w = lrelu(w.w);
  }
  const float q = a.twin_qs;
  unsigned char* dst = static_cast<unsigned char*>(a.out_twin) + o * w_esize_dev(a.twin_prec);
  if (a.twin_prec == 0) {
    *reinterpret_cast<f4*>(dst) = w * q;
  } else if (a.twin_prec == 1) {
    uint2 u;
    u.x = wpack_bf16(w.x * q, w.y * q);
    u.y = wpack_bf16(w.z * q, w.w * q);
    *reinterpret_cast<uint2*>(dst) = u;
  } else {
    *reinterpret_cast<uint32_t*>(dst) = wpack_fp8x4(w.x * q, w.y * q, w.z * q, w.w * q);
  }
}

template <int PREC>
__device__ inline f4 mfma32(const u4& alo, const u4& ahi, const u4& blo, const u4& bhi, f4 acc) {
  if constexpr (PREC == 0) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(alo[0]), __uint_as_float(blo[0]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(alo[1]), __uint_as_float(blo[1]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(alo[2]), __uint_as_float(blo[2]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(alo[3]), __uint_as_float(blo[3]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(ahi[0]), __uint_as_float(bhi[0]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(ahi[1]), __uint_as_float(bhi[1]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(ahi[2]), __uint_as_float(bhi[2]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(ahi[3]), __uint_as_float(bhi[3]), acc, 0, 0, 0);
  } else if constexpr (PREC == 1) {
    bf16x8 a0, a1, b0, b1;
    __builtin_memcpy(&a0, &alo, 16);
    __builtin_memcpy(&a1, &ahi, 16);
    __builtin_memcpy(&b0, &blo, 16);
    __builtin_memcpy(&b1, &bhi, 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
  } else {
    i8v av, bv;
    __builtin_memcpy(&av, &alo, 16);
    __builtin_memcpy(reinterpret_cast<char*>(&av) + 16, &ahi, 16);
    __builtin_memcpy(&bv, &blo, 16);
    __builtin_memcpy(reinterpret_cast<char*>(&bv) + 16, &bhi, 16);
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, 127, 0, 127);
  }
  return acc;
}

// Per-stream part of a tile (LDS).
struct WinSeg {
  const float* cache;     // current cache copy [L][cin]
  int64_t mask_x;         // local output frame t is zeroed iff t * out_den is outside [mask_x, mask_hi)
  int64_t mask_hi;
  int32_t in_start;       // first packed input frame of the stream
  int32_t out_start;      // first packed output frame (equal for stride 1)
  int32_t r0;             // first window row staged
  int32_t base;           // first LDS row of this stream's rows
  int32_t rows;
  int32_t t_lo, t_hi;     // local output frames of the stream inside the tile
};

// Per-stream part of a tile for a fused output conv (LDS): the stream's frames
// in the step, the conv's input cache (current and next copy), the user
// output and the conv's warm-up mask bound.
struct WinSeg2 {
  const float* cache2;
  float* cache2_next;
  float* out2;
  int64_t mask2_x, mask2_hi;
  int32_t T;
};

// ---- fused one-output-channel conv (see conv_win_kernel) ----
// Its output at frame t is  B + sum over taps kk of P_kk(row t - L + dil * kk),
// where P_kk(row) = sum over channels c of W[kk][c] * act(y[row][c]), added in
// tap order.  P of a row is formed with FP32 MFMA over 16-channel groups
// (tap_mfma), the groups added in order -- by the tile for its own rows, and
// by the tail launch, with the same operands, for rows of earlier steps (the
// cache) -- so a row's P has the same bits wherever it is formed, and results
// do not depend on how a stream is cut into buffers or a step into tiles.
constexpr int kOutTaps = 8;   // taps of a fused output conv, at most

// The wave's P of 16 columns over one 16-channel group, FP32 MFMA: lane
// (lr, lg) brings W[tap lr][c0 + 4 lg + j] (A) and act(y[c0 + 4 lg + j][column
// lr]) (B) at step j, and gets D[tap 4 lg + r][column lr], r = 0..3.
__device__ inline f4 tap_mfma(f4 wa, f4 y) {
  f4 d = {0.f, 0.f, 0.f, 0.f};
  d = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.x, y.x, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.y, y.y, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.z, y.z, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.w, y.w, d, 0, 0, 0);
  return d;
}

// Frames of a fused output conv left to the tail launch: the first L frames
// of a stream in the step (their taps reach the cache) and frames whose taps
// reach into the previous tile.
__device__ inline bool out_tail_frame(int32_t f, int32_t out_start, int32_t f0, int L) {
  return f - out_start < L || (out_start < f0 && f - L < f0);
}

// The epilogue of a window tile with a fused output conv.  wa: the lane's
// A operand (tap lr, channels m .. m + 3; zero beyond k).  Dynamic LDS (free
// once every wave is past the K loop): per-wave channel partials
// [WM][kOutTaps][F].
// skip_at(col): the FP32 skip row of tile column col (its channel 0).
template <int PREC, int MT, int NB, int F, class SkipAt>
__device__ inline void fused_out_epilogue(const LayerArgs& a, const f4* acc, int m, f4 bias, f4 wsc, int32_t f0,
                                          SkipAt skip_at, const WinSeg* segs, const WinSeg2* segs2,
                                          const int8_t* colseg, int n_seg, f4 wa, unsigned char* lds) {
  constexpr int WM = MT / 16;
  constexpr int WN = 4 / WM;
  constexpr int KO = kOutTaps;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lg = lane >> 4;
  const int L2 = a.oc.L, k2 = a.oc.k, d2 = a.oc.dil;
  const bool pre2 = a.oc.pre_act != 0;
  // the output conv's input channels (this conv's cout: MT, or fewer with the
  // tile's last rows padding, which stay zero)
  const int C2 = a.cout;
  const bool m_ok = m < C2;
  f4 v[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = wn * (F / WN) + nb * 16 + lr;
    const int s = colseg[col];
    v[nb] = f4{0.f, 0.f, 0.f, 0.f};
    if (s < 0 || !m_ok) continue;
    const int32_t t = f0 + col - segs[s].out_start;
    f4 x = acc[nb];
    if (PREC == 2) x = x * (wsc * a.act_scale);
    x = x + bias;
    if (a.residual) x = x + *reinterpret_cast<const f4*>(skip_at(col) + m);
    if ((int64_t)t * a.out_den < segs[s].mask_x || (int64_t)t * a.out_den >= segs[s].mask_hi) x = f4{0.f, 0.f, 0.f, 0.f};
    v[nb] = x;
  }
  __syncthreads();   // every wave is done with the staged rows and the skip rows
  float* X = reinterpret_cast<float*>(lds);   // [WM][KO][F]
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = wn * (F / WN) + nb * 16 + lr;
    const int s = colseg[col];
    if (s >= 0) {
      // the output conv's next cache: the stream's last L2 frames (raw)
      const WinSeg2& g2 = segs2[s];
      const int32_t i = f0 + col - segs[s].out_start - (g2.T - L2);
      if (i >= 0 && m_ok) gstore<f4>(g2.cache2_next + (int64_t)i * C2 + m, v[nb]);
    }
    // the wave's 16 channels of the 16 columns: D[kk][col] = sum over them of
    // W[kk][c] * act(y[c][col]) on FP32 MFMA, the accumulator layout serving
    // as the B operand (lane: channels m .. m + 3 of column col, one per step)
    const f4 y = {act(v[nb].x, pre2), act(v[nb].y, pre2), act(v[nb].z, pre2), act(v[nb].w, pre2)};
    const f4 d = tap_mfma(wa, y);
    // lane: taps 4 lg .. 4 lg + 3 of column col
    if (lg < KO / 4) {
      float* xr = X + (wm * KO + lg * 4) * F + col;
      xr[0] = d.x;
      xr[F] = d.y;
      xr[2 * F] = d.z;
      xr[3 * F] = d.w;
    }
  }
  // old cache rows that stay in the next cache of a stream of fewer than L2
  // frames (moved by the tile holding the stream's first frame)
  for (int s = 0; s < n_seg; ++s) {
    const WinSeg2& g2 = segs2[s];
    if (segs[s].t_lo != 0 || g2.T >= L2) continue;   // uniform
    for (int j = tid; j < (L2 - g2.T) * (C2 / 4); j += kThreads) {
      const int i = j / (C2 / 4);
      const int c = (j - i * (C2 / 4)) * 4;
      gstore<f4>(g2.cache2_next + (int64_t)i * C2 + c, gload<f4>(g2.cache2 + (int64_t)(g2.T + i) * C2 + c));
    }
  }
  __syncthreads();
  // P of a row: the 16-channel groups in order
  auto prow = [&](int r, int kk) {
    float p = X[kk * F + r];
#pragma unroll
    for (int w = 1; w < WM; ++w) p = p + X[(w * KO + kk) * F + r];
    return p;
  };
  if (tid < F) {
    // one lane per column: the output conv at the column's frame when all its
    // taps are on the tile's rows
    const int col = tid;
    const int s = colseg[col];
    if (s >= 0) {
      const WinSeg& g = segs[s];
      const int32_t f = f0 + col;
      const int32_t t = f - g.out_start;
      if (!out_tail_frame(f, g.out_start, f0, L2)) {
        float o = a.oc.B[0];
#pragma unroll
        for (int kk = 0; kk < KO; ++kk)
          if (kk < k2) o = o + prow(col - L2 + d2 * kk, kk);
        if (a.oc.post_act == 2) o = tanhf(o);
        if ((int64_t)t * a.out_den < segs2[s].mask2_x || (int64_t)t * a.out_den >= segs2[s].mask2_hi) o = 0.f;
        gstore<float>(segs2[s].out2 + t, o);
      }
    }
  } else if (tid - F < F) {
    // P of the column's row to out_buf where the tail launch reads it (rows
    // next to a tile boundary or among a stream's first L2 frames; P_kk at
    // float kk of the row)
    const int col = tid - F;
    const int s = colseg[col];
    if (s >= 0 && (col < L2 || col >= F - L2 || f0 + col - segs[s].out_start < L2)) {
#pragma unroll
      for (int kk = 0; kk < KO; ++kk)
        if (kk < k2) a.out_buf[(int64_t)(f0 + col) * C2 + kk] = prow(col, kk);
    }
  }
}

// MT x F tile, 4 waves: MT = 32 -> 2 x 2 waves of 16 x (F / 2); MT = 64 ->
// 4 x 1 waves of 16 x F.  A wave owns NB column blocks of 16, so F = 16 NB WN;
// all KCM 128-byte K chunks of its weight rows stay in registers.
//
// LDS: the staged window rows in operand form (activated and rounded once,
// row stride cin * ES + 16 bytes), then, for a fused residual, each column's
// skip row as raw FP32 ([F][cin + 4]), then per staged row its source pointer
// and skip slot.
//
// FUSE: a one-output-channel conv reading this layer's output (all of cout in
// one M tile: cout == MT, or 48 channels on a 64-row tile whose last 16 rows
// stay zero) runs in the epilogue, which never writes the layer's output itself.
// From the accumulators it forms each row's per-tap sums P_kk (see
// tap_partial) and finishes every frame whose taps stay on the tile's rows;
// a small tail launch finishes the rest (a stream's first L frames, and up to
// L frames after each tile boundary), reading P of the rows they need, which
// the tiles store in out_buf (the only values written there).  The tiles
// also move the output conv's input cache.
// The B operands of K chunk c for the NB column blocks of a lane: its two
// 16-byte pieces of each column's window row, element kk -> (tap, channel).
// Every read is issued before any is used (a piece past the real K reads the
// column's first row and is zeroed), so the chunk waits once for LDS instead
// of once per column block behind a branch.
// CIN > 0: the input channels are known at compile time (the tap and channel
// of a piece are then constants of c and lg); KEXACT: the K chunks hold no
// element past the real K (no piece needs zeroing).
template <int ES, int NB, int CIN = 0, bool KEXACT = false>
__device__ inline void win_chunk_reads(const FastDiv& fd_cin, int dil, int c, int lg, int Kreal, int cin, int rowb,
                                       const unsigned char* wop, const int* cb, u4* blo, u4* bhi) {
  int off[2];
  bool live[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int kk = (c * 128 + lg * 32 + p * 16) / ES;
    live[p] = KEXACT || kk < Kreal;
    const int tap = CIN > 0 ? kk / CIN : (int)fdiv(fd_cin, (uint32_t)kk);
    off[p] = live[p] ? tap * dil * rowb + (kk - tap * (CIN > 0 ? CIN : cin)) * ES : 0;
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    blo[nb] = *reinterpret_cast<const u4*>(wop + cb[nb] + off[0]);
    bhi[nb] = *reinterpret_cast<const u4*>(wop + cb[nb] + off[1]);
  }
  if constexpr (!KEXACT) {
    const u4 z = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      blo[nb] = live[0] ? blo[nb] : z;
      bhi[nb] = live[1] ? bhi[nb] : z;
    }
  }
}

// CIN > 0: an instance for cin == CIN (per-row and per-piece arithmetic on
// constants); KX: K fills the KCM chunks exactly.
template <int PREC, int MT, int NB, int KCM, bool FUSE, int CIN = 0, bool KX = false>
__global__ void __launch_bounds__(kThreads, KCM > 3 ? 4 : 5) conv_win_kernel(LayerArgs a, int n_mt, int n_nt, int Kpad, int Kreal,
                                                             int row_cap, int extra_blocks, FastDiv fd_per_ent,
                                                             FastDiv fd_ppr) {
  constexpr int WM = MT / 16;
  constexpr int WN = 4 / WM;
  constexpr int F = NB * 16 * WN;
  constexpr int ES = WPrec<PREC>::kEsize;
  constexpr int kMaxChunks = KCM;

  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ WinSeg segs[kMaxStreams];
  __shared__ WinSeg2 segs2[FUSE ? kMaxStreams : 1];
  __shared__ int32_t colbase[F];
  __shared__ int8_t colseg[F];
  __shared__ int8_t colkeep[F];   // per column: -1 past the step, 0 zeroed by a mask, 1 kept

  const int tid = threadIdx.x;
  const int32_t n_tiles = n_mt * n_nt;
  const int32_t bid = blockIdx.x;

  // ---- cache update blocks (after the tiles): new cache = last L window rows,
  // 4 channels per item ----
  if (bid >= n_tiles) {
    const int32_t per_ent = a.L * a.cin / 4;
    const int32_t total = step_ents(a) * per_ent;
    for (int32_t j = (bid - n_tiles) * kThreads + tid; j < total; j += extra_blocks * kThreads) {
      const int ei = (int)fdiv(fd_per_ent, (uint32_t)j);
      const int32_t rem = (j - ei * per_ent) * 4;
      const int32_t i = (int32_t)fdiv(a.fd_cin, (uint32_t)rem);
      const int ci = rem - i * a.cin;
      const Entry e = load_entry(a.ents + ei);
      const int32_t row = in_frames(a, e.T) + i;
      const float* src = row < a.L ? e.state + a.state_off + (int64_t)e.parity * a.state_len + (int64_t)row * a.cin + ci
                                   : a.in_buf + ((int64_t)in_frames(a, e.off) + row - a.L) * a.cin + ci;
      gstore<f4>(e.state + a.state_off + (int64_t)(1 - e.parity) * a.state_len + (int64_t)i * a.cin + ci,
                 gload<f4>(src));
    }
    return;
  }

  const int mt = (int)((uint32_t)bid % (uint32_t)n_mt);
  const int32_t nt = (int32_t)((uint32_t)bid / (uint32_t)n_mt);
  const int m0 = mt * MT;
  const int32_t f0 = nt * F;
  const TileSpan sp = tile_span(a, f0, F);
  if (f0 >= sp.n_cols) return;          // the grid may be sized for a larger step
  const int32_t f_last = sp.f_last;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lg = lane >> 4;
  const int n_chunks = Kpad * ES / 128;
  const bool pre = a.pre_act != 0;
  const float qs = PREC == 2 ? 1.0f / a.act_scale : 1.0f;
  const int cin = CIN > 0 ? CIN : a.cin;
  const int rowb = cin * ES + 16;         // operand row stride (bytes), padded against bank conflicts
  const int skipf = cin + 4;              // skip row stride (floats)
  unsigned char* wop = lds;
  float* wskip = reinterpret_cast<float*>(lds + row_cap * rowb);
  const float** rsrc = reinterpret_cast<const float**>(lds + row_cap * rowb + F * skipf * 4);
  int32_t* rskip = reinterpret_cast<int32_t*>(rsrc + row_cap);

  // weights of the wave's 16 rows, all chunks (independent of the columns: issued first)
  u4 alo[kMaxChunks], ahi[kMaxChunks];
  {
    const unsigned char* wrow = static_cast<const unsigned char*>(a.W) +
                                (int64_t)(m0 + wm * 16 + lr) * (Kpad * ES) + lg * 32;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      if (c < n_chunks) {
        alo[c] = *reinterpret_cast<const u4*>(wrow + c * 128);
        ahi[c] = *reinterpret_cast<const u4*>(wrow + c * 128 + 16);
      }
    }
  }
  // epilogue operands of the lane's rows m .. m + 3
  const int m = m0 + wm * 16 + lg * 4;
  const bool m_ok = m < a.cout;
  const f4 bias = m_ok ? *reinterpret_cast<const f4*>(a.B + m) : f4{0.f, 0.f, 0.f, 0.f};
  const f4 wsc = (PREC == 2 && m_ok) ? *reinterpret_cast<const f4*>(a.wscale + m) : f4{1.f, 1.f, 1.f, 1.f};

  // fused output conv: the lane's A operand of its per-tap sums (tap lr,
  // channels m .. m + 3), loaded now and held through the K loop
  f4 wa2 = {0.f, 0.f, 0.f, 0.f};
  if constexpr (FUSE) {
    const int m2 = wm * 16 + lg * 4;
    if (lr < a.oc.k && m2 < a.cout) wa2 = *reinterpret_cast<const f4*>(a.oc.W + lr * a.cout + m2);
  }

  // ---- the streams of the tile: lane s of every wave forms stream s's
  // record; wave 0 publishes them ----
  const int e_first = sp.e0;
  const int n_seg = sp.n_seg;
  // the host sizes tiles so that these hold; never index LDS beyond them
  if (n_seg > kMaxStreams) return;
  int32_t R = 0;
  {
    const Entry e = load_entry(a.ents + e_first + min(lane, n_seg - 1));
    WinSeg g{};
    if (lane < n_seg) {
      g.cache = e.state + a.state_off + (int64_t)e.parity * a.state_len;
      g.mask_x = mask_lo(e, a.delay, a.out_num, a.out_den);
      g.mask_hi = mask_hi(e, a.delay, a.out_num, a.out_den);
      g.in_start = in_frames(a, e.off);
      g.out_start = out_frames(a, e.off);
      g.t_lo = lane == 0 ? f0 - g.out_start : 0;
      g.t_hi = lane == n_seg - 1 ? f_last - g.out_start : out_frames(a, e.T) - 1;
      g.r0 = g.t_lo;
      g.rows = g.t_hi - g.t_lo + 1 + a.L;
    }
    // each stream's first LDS row: the rows of the streams before it
    for (int s = 0; s < n_seg; ++s) {
      const int32_t r = __shfl(g.rows, s);
      g.base += s < lane ? r : 0;
      R += r;
    }
    if (wave == 0 && lane < n_seg) {
      segs[lane] = g;
      if constexpr (FUSE) {
        WinSeg2 g2;
        g2.T = out_frames(a, e.T);
        g2.cache2 = e.state + a.oc.state_off + (int64_t)e.parity * a.oc.state_len;
        g2.cache2_next = e.state + a.oc.state_off + (int64_t)(1 - e.parity) * a.oc.state_len;
        g2.out2 = e.out;
        g2.mask2_x = mask_lo(e, a.oc.delay, a.out_num, a.out_den);
        g2.mask2_hi = mask_hi(e, a.oc.delay, a.out_num, a.out_den);
        segs2[lane] = g2;
      }
    }
  }
  if (R > row_cap) return;
  __syncthreads();

  // column -> stream, and the LDS row of its window row t
  if (tid < F) {
    const int32_t f = f0 + tid;
    int s = 0;
    int8_t keep = -1;
    if (f <= f_last) {
      while (s + 1 < n_seg && segs[s + 1].out_start <= f) ++s;
      colbase[tid] = segs[s].base + (f - segs[s].out_start - segs[s].r0);
      const int64_t x = (int64_t)(f - segs[s].out_start) * a.out_den;
      keep = x < segs[s].mask_x || x >= segs[s].mask_hi ? 0 : 1;
    } else {
      colbase[tid] = 0;
      s = -1;
    }
    colseg[tid] = (int8_t)s;
    colkeep[tid] = keep;
  }

  // each staged row's source (cache or input) and, for a fused residual, the
  // column whose skip row it is (-1: none); one stream search per row
  for (int32_t j = tid; j < R; j += kThreads) {
    int s = 0;
    while (s + 1 < n_seg && segs[s + 1].base <= j) ++s;
    const WinSeg& g = segs[s];
    const int32_t r = g.r0 + (j - g.base);
    rsrc[j] = r < a.L ? g.cache + (int64_t)r * cin : a.in_buf + ((int64_t)g.in_start + r - a.L) * cin;
    const int32_t t = r - a.skip_off;
    rskip[j] = (a.residual && t >= g.t_lo && t <= g.t_hi) ? g.out_start + t - f0 : -1;
  }
  __syncthreads();

  // ---- stage the window rows: operand form, plus the raw skip rows ----
  {
    const int ppr = cin >> 2;              // 16-byte FP32 source pieces per row
    const int32_t n_pieces = R * ppr;
    constexpr int SB = kStageBatch;
    for (int32_t i0 = 0; i0 < n_pieces; i0 += kThreads * SB) {
      // all loads of the batch first (one round trip), then the LDS stores;
      // the piece's row and stream are recomputed for the stores to keep
      // registers for the loads only
      f4 v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int32_t idx = i0 + u * kThreads + tid;
        v[u] = f4{0.f, 0.f, 0.f, 0.f};
        if (idx < n_pieces) {
          const int32_t j = CIN > 0 ? idx / (CIN / 4) : (int32_t)fdiv(fd_ppr, (uint32_t)idx);
          const int pc = idx - j * ppr;
          v[u] = gload<f4>(rsrc[j] + pc * 4);
        }
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int32_t idx = i0 + u * kThreads + tid;
        if (idx >= n_pieces) continue;
        const int32_t j = CIN > 0 ? idx / (CIN / 4) : (int32_t)fdiv(fd_ppr, (uint32_t)idx);
        const int pc = idx - j * ppr;
        const f4 x = v[u];
        unsigned char* dst = wop + j * rowb + pc * 4 * ES;
        if constexpr (PREC == 0) {
          *reinterpret_cast<f4*>(dst) = f4{act(x.x, pre), act(x.y, pre), act(x.z, pre), act(x.w, pre)};
        } else if constexpr (PREC == 1) {
          uint2 w;
          w.x = wpack_bf16(act(x.x, pre), act(x.y, pre));
          w.y = wpack_bf16(act(x.z, pre), act(x.w, pre));
          *reinterpret_cast<uint2*>(dst) = w;
        } else {
          *reinterpret_cast<uint32_t*>(dst) =
              wpack_fp8x4(act(x.x, pre) * qs, act(x.y, pre) * qs, act(x.z, pre) * qs, act(x.w, pre) * qs);
        }
        const int32_t sk = rskip[j];
        if (sk >= 0) *reinterpret_cast<f4*>(&wskip[sk * skipf + pc * 4]) = x;
      }
    }
  }
  __syncthreads();

  // ---- K loop: B operands read straight from the staged rows ----
  int cb[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) cb[nb] = colbase[wn * (F / WN) + nb * 16 + lr] * rowb;
  f4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    if (c < n_chunks) {
      u4 blo[NB], bhi[NB];
      win_chunk_reads<ES, NB, CIN, KX>(a.fd_cin, a.dil, c, lg, Kreal, cin, rowb, wop, cb, blo, bhi);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma32<PREC>(alo[c], ahi[c], blo[nb], bhi[nb], acc[nb]);
    }
  }

  if constexpr (FUSE) {
    fused_out_epilogue<PREC, MT, NB, F>(
        a, acc, m, bias, wsc, f0, [&](int col) { return wskip + col * skipf; }, segs, segs2, colseg, n_seg, wa2, lds);
    return;
  }

  // ---- epilogue: lane holds rows m .. m + 3 of column col for each block ----
  if (!m_ok) return;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = wn * (F / WN) + nb * 16 + lr;
    const int keep = colkeep[col];
    if (keep < 0) continue;
    const int32_t f = f0 + col;
    f4 v = acc[nb];
    if (PREC == 2) v = v * (wsc * a.act_scale);
    v = v + bias;
    if (a.residual) v = v + *reinterpret_cast<const f4*>(&wskip[col * skipf + m]);
    if (!keep) v = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t o = (int64_t)f * a.cout + m;
    if (!a.twin_only) gstore<f4>(a.out_buf + o, v);
    if (a.out_twin) store_twin(a, o, v);
  }
}

// ---- a window conv with the transposed conv before it in the same launch ----
//
// The residual conv's input x is the output of a transposed conv (ratio r,
// kernel 2r) that nothing else reads.  Each tile computes the x frames its
// window needs -- its own frames plus the L frames before them -- from the
// transposed conv's input (operand form, written by that conv's producer),
// so x never goes to memory.  Frame q * r + phi of x is the transposed-conv
// GEMM column q, row phi * cout + co, over K = [input q - 1 | input q]
// (the chunks and MFMA instructions of its own launch); column q = 0 of a
// buffer starts from the FP32 carry, and the tile that holds a stream's last
// frame also runs column q = T_in (the carry of the next buffer).  The
// values of x, its rounding into the conv's operand and the conv itself are
// bit for bit those of the two separate launches.
//
// LDS: region X holds the transposed conv's input frames, each staged once
// (column q reads rows q - 1 and q as its two K halves) and, once every wave
// is past those MFMAs, x's window rows in FP32 (the residual skip); region O
// the window rows in operand form.  The conv's cache is the last L frames of
// x: written by the tiles that own them (every stream brings at least L
// frames, so no old cache row survives).  Every global load that does not
// depend on the staged data (both layers' weights, biases and scales, the
// cache rows of the window) is issued before the staging barrier.

// Per-stream part of a fused tile (LDS): the transposed conv's side.
struct CtSeg {
  const float* carry;      // current carry copy [r * cout]
  float* carry_next;
  float* cache_next;       // the conv's next cache copy [L][cout]
  int64_t mask_lo, mask_hi;   // x frame t is zeroed iff t * den is outside [mask_lo, mask_hi)
  int32_t in_start;        // first packed frame of the transposed conv's input
  int32_t Tin;             // its input frames of the stream
  int32_t T;               // x frames of the stream
  int32_t col0, qa, nq;    // first column of the stream, its first q, q columns (carry column after them)
  int32_t carry_col;       // 1: the tile computes the carry column
  int32_t xrow0;           // staged row of input frame qa - 1
};

// MBW: transposed-conv M blocks of 16 rows per wave (r * cout / 64); NCB:
// 16-column blocks of transposed-conv columns per tile, at most.
// KCM: the conv's K chunks (exactly).
template <int PREC, int MT, int NB, int KCM, int KCT, int MBW, int NCB>
__global__ void __launch_bounds__(kThreads, 5) convt_win_kernel(LayerArgs a, int n_nt, int Kpad, int Kreal,
                                                                int row_cap, int xrow_cap, int stash_cap) {
  constexpr int WM = MT / 16;
  constexpr int WN = 4 / WM;
  constexpr int F = NB * 16 * WN;
  constexpr int ES = WPrec<PREC>::kEsize;
  constexpr int EPP = 16 / ES;                 // operand elements per 16-byte piece
  constexpr int HB = KCT * 64;                 // bytes of one input frame in operand form (half of K)
  constexpr int XROW = HB + 16;                // staged input row stride (padded)
  constexpr int CPH = KCT / 2;                 // K chunks per half
  constexpr int PPR = HB / 16;                 // 16-byte pieces per staged row
  constexpr int CPRE = 2;                      // cache-row pieces per thread (the host bounds L)
  constexpr int XP = ((NCB * 16 + kMaxStreams) * PPR + kThreads - 1) / kThreads;   // staged pieces per thread

  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ WinSeg segs[kMaxStreams];
  __shared__ CtSeg csegs[kMaxStreams];
  __shared__ int32_t colbase[F];
  __shared__ int8_t colseg[F];
  __shared__ int8_t colkeep[F];   // per column: -1 past the step, 0 zeroed by a mask, 1 kept
  __shared__ int8_t ccol_seg[NCB * 16];
  __shared__ int32_t ccol_q[NCB * 16];
  __shared__ int32_t ccol_x[NCB * 16];
  // per transposed-conv column (x frames t = q * r + phi, phi < r): {q * r
  // (-1: the carry column), LDS row of phi = 0, and as byte pairs [lo, end)
  // of phi: the phases whose window rows are staged, those kept by the masks,
  // those written to the conv's next cache}
  __shared__ i4 ccol_rec[NCB * 16];

  const int tid = threadIdx.x;
  const int32_t nt = blockIdx.x;
  if (nt >= n_nt) return;
  const int32_t f0 = nt * F;
  const TileSpan sp = tile_span(a, f0, F);
  if (f0 >= sp.n_cols) return;          // the grid may be sized for a larger step
  const int32_t f_last = sp.f_last;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const bool pre = a.pre_act != 0;
  const float qs = PREC == 2 ? 1.0f / a.act_scale : 1.0f;
  const int L = a.L;
  const int R = a.ct.r;
  const int rowb = MT * ES + 16;              // operand row stride (bytes)
  constexpr int XF = MT;                      // FP32 row stride (floats): unpadded, for 5 workgroups per CU
  unsigned char* X = lds;
  float* xf = reinterpret_cast<float*>(lds);  // x rows in FP32, [row][XF] (after the transposed-conv MFMAs)
  // the window's cache rows in FP32 until X is free (stash_cap f4 pieces)
  f4* stash = reinterpret_cast<f4*>(lds + (size_t)max(xrow_cap * XROW, row_cap * XF * 4));
  unsigned char* wop = lds + (size_t)max(xrow_cap * XROW, row_cap * XF * 4) + (size_t)stash_cap * 16;

  // both layers' weights, biases and scales (independent of the columns)
  const int wm = wave % WM, wn = wave / WM;
  u4 alo[KCM], ahi[KCM];
  {
    const unsigned char* wrow = static_cast<const unsigned char*>(a.W) + (int64_t)(wm * 16 + lr) * (Kpad * ES) + lg * 32;
#pragma unroll
    for (int c = 0; c < KCM; ++c) {
      alo[c] = *reinterpret_cast<const u4*>(wrow + c * 128);
      ahi[c] = *reinterpret_cast<const u4*>(wrow + c * 128 + 16);
    }
  }
  const int m_cv = wm * 16 + lg * 4;
  const f4 bias = *reinterpret_cast<const f4*>(a.B + m_cv);
  const f4 wsc = PREC == 2 ? *reinterpret_cast<const f4*>(a.wscale + m_cv) : f4{1.f, 1.f, 1.f, 1.f};

  // ---- the streams of the tile: lane s of every wave forms stream s's
  // records; wave 0 publishes them ----
  const int e_first = sp.e0;
  const int n_seg = sp.n_seg;
  // the host sizes tiles so that these hold; never index LDS beyond them
  if (n_seg > kMaxStreams) return;
  int32_t n_rows = 0, n_ccol = 0, n_cp = 0;
  {
    WinSeg g{};
    CtSeg c{};
    int32_t ncols = 0, cpieces = 0;
    const Entry e = load_entry(a.ents + e_first + min(lane, n_seg - 1));
    if (lane < n_seg) {
      g.cache = e.state + a.state_off + (int64_t)e.parity * a.state_len;
      g.mask_x = mask_lo(e, a.delay, a.out_num, a.out_den);
      g.mask_hi = mask_hi(e, a.delay, a.out_num, a.out_den);
      g.in_start = in_frames(a, e.off);
      g.out_start = out_frames(a, e.off);
      const int32_t T = out_frames(a, e.T);
      g.t_lo = lane == 0 ? f0 - g.out_start : 0;
      g.t_hi = lane == n_seg - 1 ? f_last - g.out_start : T - 1;
      g.r0 = g.t_lo;
      g.rows = g.t_hi - g.t_lo + 1 + L;
      c.carry = e.state + a.ct.state_off + (int64_t)e.parity * a.ct.state_len;
      c.carry_next = e.state + a.ct.state_off + (int64_t)(1 - e.parity) * a.ct.state_len;
      c.cache_next = e.state + a.state_off + (int64_t)(1 - e.parity) * a.state_len;
      // x is this layer's input: its mask runs at the input rate
      c.mask_lo = mask_lo(e, a.ct.delay, a.in_num, a.in_den);
      c.mask_hi = mask_hi(e, a.ct.delay, a.in_num, a.in_den);
      c.in_start = (int32_t)fdiv(a.ct.fd_in_den, (uint32_t)e.off * a.ct.in_num);
      c.Tin = (int32_t)fdiv(a.ct.fd_in_den, (uint32_t)e.T * a.ct.in_num);
      c.T = T;
      // x frames of the window: [max(0, t_lo - L), t_hi] -> q in [qa, t_hi / r]
      const int32_t ta = max(0, g.t_lo - L);
      c.qa = ta / R;
      c.nq = g.t_hi / R - c.qa + 1;
      c.carry_col = g.t_hi == T - 1 ? 1 : 0;
      ncols = c.nq + c.carry_col;
      cpieces = max(0, min(L - g.r0, g.rows)) * (MT / 4);
    }
    // each stream's first window row, first column and first staged row
    // (one more staged row than columns per stream): sums over the streams before it
    for (int s = 0; s < n_seg; ++s) {
      const int32_t r = __shfl(g.rows, s);
      const int32_t nc = __shfl(ncols, s);
      g.base += s < lane ? r : 0;
      c.col0 += s < lane ? nc : 0;
      n_rows += r;
      n_ccol += nc;
      n_cp += __shfl(cpieces, s);
    }
    c.xrow0 = c.col0 + lane;
    if (wave == 0 && lane < n_seg) {
      segs[lane] = g;
      csegs[lane] = c;
    }
  }
  if (n_rows > row_cap || n_ccol > NCB * 16 || n_ccol + n_seg > xrow_cap || n_cp > stash_cap ||
      n_cp > CPRE * kThreads)
    return;
  __syncthreads();

  // the transposed conv's weights, bias and scales (r * MT = 64 * MBW rows: M
  // block wave + 4 mi), issued with the staging loads below
  u4 tlo[MBW][KCT], thi[MBW][KCT];
  f4 ct_bias[MBW], ct_ws[MBW];
#pragma unroll
  for (int mi = 0; mi < MBW; ++mi) {
    const int mb = wave + 4 * mi;
    const unsigned char* wrow =
        static_cast<const unsigned char*>(a.ct.W) + (int64_t)(mb * 16 + lr) * (a.ct.Kpad * ES) + lg * 32;
#pragma unroll
    for (int c = 0; c < KCT; ++c) {
      tlo[mi][c] = *reinterpret_cast<const u4*>(wrow + c * 128);
      thi[mi][c] = *reinterpret_cast<const u4*>(wrow + c * 128 + 16);
    }
    const int m = mb * 16 + lg * 4;
    ct_bias[mi] = *reinterpret_cast<const f4*>(a.ct.B + (m - (m / MT) * MT));
    ct_ws[mi] = PREC == 2 ? *reinterpret_cast<const f4*>(a.ct.wscale + m) : f4{1.f, 1.f, 1.f, 1.f};
  }

  // ---- transposed-conv input frames qa - 1 .. qa + nq - 1 (+1 with the carry column), each once, and
  // the window's cache rows (rows below L): every load of the tile in flight at once ----
  u4 xv[XP];
  f4 cpre[CPRE];
  int32_t cdst[CPRE];
  {
    const int32_t n_pieces = (n_ccol + n_seg) * PPR;
    const unsigned char* tin = static_cast<const unsigned char*>(a.ct.in_twin);
#pragma unroll
    for (int p = 0; p < XP; ++p) {
      const int32_t idx = tid + p * kThreads;
      xv[p] = u4{0u, 0u, 0u, 0u};
      if (idx < n_pieces) {
        const int xr = idx / PPR;
        const int pc = idx - xr * PPR;
        int s = 0;
        while (s + 1 < n_seg && csegs[s + 1].xrow0 <= xr) ++s;
        const int row = csegs[s].qa - 1 + (xr - csegs[s].xrow0);
        const int ci = pc * EPP;
        if (ci < a.ct.cin && row >= 0 && row < csegs[s].Tin)
          xv[p] = gload<u4>(tin + ((int64_t)(csegs[s].in_start + row) * a.ct.cin + ci) * ES);
      }
    }
#pragma unroll
    for (int p = 0; p < CPRE; ++p) {
      cdst[p] = -1;
      int32_t idx = tid + p * kThreads;
      for (int s = 0; s < n_seg; ++s) {
        const WinSeg& g = segs[s];
        const int32_t n = max(0, min(L - g.r0, g.rows)) * (MT / 4);
        if (idx < n) {
          const int32_t i = idx / (MT / 4);
          const int ch = (idx - i * (MT / 4)) * 4;
          cpre[p] = gload<f4>(g.cache + (int64_t)(g.r0 + i) * MT + ch);
          cdst[p] = (g.base + i) * MT + ch;
          break;
        }
        idx -= n;
      }
    }
#pragma unroll
    for (int p = 0; p < XP; ++p) {
      const int32_t idx = tid + p * kThreads;
      if (idx < n_pieces) *reinterpret_cast<u4*>(X + (idx / PPR) * XROW + (idx % PPR) * 16) = xv[p];
    }
#pragma unroll
    for (int p = 0; p < CPRE; ++p)
      if (cdst[p] >= 0) stash[tid + p * kThreads] = cpre[p];
  }
  // column -> stream and window row (the conv), transposed-conv column -> (stream, q, staged row)
  if (tid < F) {
    const int32_t f = f0 + tid;
    int s = 0;
    int8_t keep = -1;
    if (f <= f_last) {
      while (s + 1 < n_seg && segs[s + 1].out_start <= f) ++s;
      colbase[tid] = segs[s].base + (f - segs[s].out_start - segs[s].r0);
      const int64_t x = (int64_t)(f - segs[s].out_start) * a.out_den;
      keep = x < segs[s].mask_x || x >= segs[s].mask_hi ? 0 : 1;
    } else {
      colbase[tid] = 0;
      s = -1;
    }
    colseg[tid] = (int8_t)s;
    colkeep[tid] = keep;
  }
  for (int j = tid; j < NCB * 16; j += kThreads) {
    int s = -1, q = 0, x = 0;
    if (j < n_ccol) {
      s = 0;
      while (s + 1 < n_seg && csegs[s + 1].col0 <= j) ++s;
      q = csegs[s].qa + (j - csegs[s].col0);   // the carry column: q = qa + nq = T_in
      x = csegs[s].xrow0 + (j - csegs[s].col0);
    }
    ccol_seg[j] = (int8_t)s;
    ccol_q[j] = q;
    ccol_x[j] = x;
    i4 rec = {-1, 0, 0, 0};
    if (s >= 0) {
      const CtSeg& c = csegs[s];
      const WinSeg& g = segs[s];
      if (q != c.Tin) {
        // a range [lo, end) of x frames as a range of phases of this column
        const int32_t t0 = q * R;
        auto ph = [&](int32_t lo, int32_t end) {
          const int32_t a0 = min(max(lo - t0, 0), R), a1 = min(max(end - t0, 0), R);
          return (a0 & 0xff) | (a1 & 0xff) << 8;
        };
        const int32_t staged = ph(g.r0 - L, g.r0 - L + g.rows);
        const int32_t kept = ph(ceil_frames(c.mask_lo, a.in_den), ceil_frames(c.mask_hi, a.in_den));
        const int32_t cached = ph(max(c.T - L, g.t_lo), g.t_hi + 1);
        rec = i4{t0, g.base + L - g.r0 + t0, staged | kept << 16, cached};
      }
    }
    ccol_rec[j] = rec;
  }
  __syncthreads();

  // ---- transposed-conv MFMAs: the wave's M blocks x every column block ----
  const int ncb = (n_ccol + 15) / 16;
  f4 cacc[MBW][NCB];
#pragma unroll
  for (int mi = 0; mi < MBW; ++mi) {
    const int m = (wave + 4 * mi) * 16 + lg * 4;   // the lane's rows m .. m + 3 (accumulator layout)
#pragma unroll
    for (int nc = 0; nc < NCB; ++nc) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      if (nc < ncb) {
        const int col = nc * 16 + lr;
        // column q = 0 of a buffer starts from the carry
        if (col < n_ccol && ccol_q[col] == 0) {
          const CtSeg& c = csegs[ccol_seg[col]];
          if (c.Tin > 0) acc = gload<f4>(c.carry + m);
        }
        const unsigned char* xb = X + ccol_x[col] * XROW + lg * 32;
#pragma unroll
        for (int c = 0; c < KCT; ++c) {
          const unsigned char* p = xb + (c / CPH) * XROW + (c % CPH) * 128;
          acc = mfma32<PREC>(tlo[mi][c], thi[mi][c], *reinterpret_cast<const u4*>(p),
                             *reinterpret_cast<const u4*>(p + 16), acc);
        }
      }
      cacc[mi][nc] = acc;
    }
  }
  __syncthreads();   // every wave is past the staged input: X now takes x's FP32 rows

  // ---- x: bias, mask, FP32 rows, operand rows, the conv's next cache, the next carry ----
#pragma unroll
  for (int mi = 0; mi < MBW; ++mi) {
    const int m = (wave + 4 * mi) * 16 + lg * 4;
    const int phi = m / MT;
    const int co = m - phi * MT;
#pragma unroll
    for (int nc = 0; nc < NCB; ++nc) {
      const int col = nc * 16 + lr;
      if (nc >= ncb || col >= n_ccol) continue;
      const i4 rec = ccol_rec[col];
      if (rec.x < 0) {
        // the carry of the next buffer, in accumulator units
        gstore<f4>(csegs[ccol_seg[col]].carry_next + m, cacc[mi][nc]);
        continue;
      }
      f4 v = cacc[mi][nc];
      if (PREC == 2) v = v * (ct_ws[mi] * a.ct.act_scale);
      v = v + ct_bias[mi];
      const int32_t t = rec.x + phi;           // x frame of the stream
      if (phi < ((rec.z >> 16) & 0xff) || phi >= (rec.z >> 24)) v = f4{0.f, 0.f, 0.f, 0.f};   // masks
      if (phi >= (rec.z & 0xff) && phi < ((rec.z >> 8) & 0xff)) {   // its window row t + L is staged
        const int32_t j = rec.y + phi;
        *reinterpret_cast<f4*>(xf + (size_t)j * XF + co) = v;
        unsigned char* dst = wop + (size_t)j * rowb + co * ES;
        if constexpr (PREC == 1) {
          uint2 u;
          u.x = wpack_bf16(act(v.x, pre), act(v.y, pre));
          u.y = wpack_bf16(act(v.z, pre), act(v.w, pre));
          *reinterpret_cast<uint2*>(dst) = u;
        } else {
          *reinterpret_cast<uint32_t*>(dst) =
              wpack_fp8x4(act(v.x, pre) * qs, act(v.y, pre) * qs, act(v.z, pre) * qs, act(v.w, pre) * qs);
        }
      }
      // the conv's next cache: the stream's last L frames of x, by the tile that owns them
      if (phi >= (rec.w & 0xff) && phi < (rec.w >> 8)) {
        const CtSeg& c = csegs[ccol_seg[col]];
        gstore<f4>(c.cache_next + (int64_t)(t - (c.T - L)) * MT + co, v);
      }
    }
  }
  // window rows from the conv's cache (rows below L)
#pragma unroll
  for (int p = 0; p < CPRE; ++p) {
    if (cdst[p] < 0) continue;
    const f4 v = stash[tid + p * kThreads];
    const int32_t jr = cdst[p] / MT;
    const int ch = cdst[p] - jr * MT;
    *reinterpret_cast<f4*>(xf + (size_t)jr * XF + ch) = v;
    unsigned char* dst = wop + (size_t)jr * rowb + ch * ES;
    if constexpr (PREC == 1) {
      uint2 u;
      u.x = wpack_bf16(act(v.x, pre), act(v.y, pre));
      u.y = wpack_bf16(act(v.z, pre), act(v.w, pre));
      *reinterpret_cast<uint2*>(dst) = u;
    } else {
      *reinterpret_cast<uint32_t*>(dst) =
          wpack_fp8x4(act(v.x, pre) * qs, act(v.y, pre) * qs, act(v.z, pre) * qs, act(v.w, pre) * qs);
    }
  }
  __syncthreads();

  // ---- the conv: B operands from the staged rows, the skip from x's FP32 rows ----
  const int m = m_cv;
  constexpr int n_chunks = KCM;
  int cb[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) cb[nb] = colbase[wn * (F / WN) + nb * 16 + lr] * rowb;
  f4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < KCM; ++c) {
    if (c < n_chunks) {
      u4 blo[NB], bhi[NB];
      win_chunk_reads<ES, NB, MT>(a.fd_cin, a.dil, c, lg, Kreal, MT, rowb, wop, cb, blo, bhi);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma32<PREC>(alo[c], ahi[c], blo[nb], bhi[nb], acc[nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = wn * (F / WN) + nb * 16 + lr;
    const int keep = colkeep[col];
    if (keep < 0) continue;
    const int32_t f = f0 + col;
    f4 v = acc[nb];
    if (PREC == 2) v = v * (wsc * a.act_scale);
    v = v + bias;
    if (a.residual) v = v + *reinterpret_cast<const f4*>(xf + (size_t)(colbase[col] + a.skip_off) * XF + m);
    if (!keep) v = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t o = (int64_t)f * a.cout + m;
    if (!a.twin_only) gstore<f4>(a.out_buf + o, v);
    if (a.out_twin) store_twin(a, o, v);
  }
}

// ---- two residual window convs in one launch ----
//
// Conv A's output x1 has one reader, conv B (the next residual conv of the
// stack).  Each tile of B's output frames computes the x1 frames its window
// needs -- its own frames and the L_B before them, back to the start of the
// stream's buffer -- from A's window, so x1 never goes to memory; B's window
// rows before the buffer come from B's cache.  x1, its rounding into B's
// operand and B itself are bit for bit those of the two launches (the same K
// chunks, MFMA instructions and epilogue order).
//
// LDS: region 1 holds A's window rows in operand form and, once every wave is
// past A's MFMAs, B's window rows in FP32 (B's skip); then B's cache rows in
// FP32 until region 1 is free, B's window rows in operand form and A's row
// sources.  A's skip values go to registers with the staging loads.  A's next
// cache (its last L_A window rows) is written by the blocks after the tiles,
// B's (the stream's last L_B frames of x1) by the tiles that own those frames
// (every stream brings at least L_B frames, so no old cache row survives).

// Per-stream part of a pair tile (LDS): conv A's side.
struct PairSeg {
  const float* cache_a;    // A's current cache [L_A][C]
  float* cache_b_next;     // B's next cache copy [L_B][C]
  int64_t mask_lo, mask_hi;   // x1 frame u is zeroed iff u * den is outside [mask_lo, mask_hi)
  int32_t in_start;        // first packed frame of A's input
  int32_t T;               // frames of the stream
  int32_t ta;              // first x1 frame the tile computes
  int32_t acol0;           // its A column
  int32_t abase;           // LDS row of A's window row ta
};

// MT: the rows of the M tile; CH: the channels of both convs (MT, or 48 on a
// 64-row tile whose last 16 rows are padding: their lanes write nothing);
// waves split B's tile as the window kernel does (WM row blocks x WN column
// halves) and A's columns the same way.  NCBA: A column blocks a tile holds
// at most.  FUSE: B computes a one-output-channel conv in its epilogue
// (fused_out_epilogue).
template <int PREC, int MT, int NB, int KCM, int NCBA, bool FUSE, int CH = MT>
__global__ void __launch_bounds__(kThreads, 4) conv_pair_kernel(LayerArgs a, int n_nt, int Kpad, int Kreal,
                                                                int row_cap, int arow_cap, int stash_cap,
                                                                int extra_blocks, FastDiv fd_per_ent) {
  constexpr int WM = MT / 16;
  constexpr int WN = 4 / WM;
  constexpr int C = CH;                        // channels of both convs
  static_assert(C <= MT && C % 16 == 0, "the channels fill whole 16-row blocks of the tile");
  constexpr int F = NB * 16 * WN;
  constexpr int NCW = NCBA / WN;               // A column blocks of a wave
  static_assert(NCW % 2 == 0, "two groups of column blocks per wave");
  static_assert(F * (C + 4) < 0x7fff, "skip-row offsets in 15 bits");
  constexpr int ES = WPrec<PREC>::kEsize;
  constexpr int ROWB = C * ES + 16;            // operand row stride (bytes), padded against bank conflicts
  constexpr int XF = C + 4;                    // FP32 row stride (floats), padded likewise
  constexpr int PPR = C / 4;                   // 16-byte FP32 pieces per row
  constexpr int CPRE = 2;                      // B cache-row pieces per thread (the host bounds L_B)
  constexpr int NCOL = NCBA * 16;              // A columns a tile holds at most
  constexpr int SB = kStageBatch;
  constexpr bool KX = 3 * C * ES == KCM * 128; // K = 3 C fills the chunks (BF16)

  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ WinSeg segs[kMaxStreams];
  __shared__ PairSeg psegs[kMaxStreams];
  __shared__ WinSeg2 segs2[FUSE ? kMaxStreams : 1];
  __shared__ int32_t colbase[F];
  __shared__ int8_t colkeep[F];
  __shared__ int8_t colseg[F];
  __shared__ int32_t acb[NCOL];                // A column: LDS row of its first window row
  __shared__ int32_t ajb[NCOL];                // A column: LDS row of its frame in B's window
  __shared__ int16_t aslot[NCOL];              // A column: the B column whose skip row it is (-1: none)
  __shared__ int8_t aflag[NCOL];               // bit 0: kept by A's masks; bit 1: a row of B's next cache
  __shared__ const float* askip[NCOL];         // A column: its skip row (A's cache or input)
  __shared__ float* anext[NCOL];               // A column: its row of B's next cache

  const int tid = threadIdx.x;
  const int32_t bid = blockIdx.x;
  const int LA = a.pa.L, LB = a.L;

  // ---- A's cache update blocks (after the tiles): A's next cache = its last
  // L_A window rows, 4 channels per item ----
  if (bid >= n_nt) {
    const int32_t per_ent = LA * C / 4;
    const int32_t total = step_ents(a) * per_ent;
    for (int32_t j = (bid - n_nt) * kThreads + tid; j < total; j += extra_blocks * kThreads) {
      const int ei = (int)fdiv(fd_per_ent, (uint32_t)j);
      const int32_t rem = (j - ei * per_ent) * 4;
      const int32_t i = rem / C;
      const int ci = rem - i * C;
      const Entry e = load_entry(a.ents + ei);
      const int32_t row = in_frames(a, e.T) + i;
      const float* src = row < LA ? e.state + a.pa.state_off + (int64_t)e.parity * a.pa.state_len + (int64_t)row * C + ci
                                  : a.pa.in_buf + ((int64_t)in_frames(a, e.off) + row - LA) * C + ci;
      gstore<f4>(e.state + a.pa.state_off + (int64_t)(1 - e.parity) * a.pa.state_len + (int64_t)i * C + ci,
                 gload<f4>(src));
    }
    return;
  }

  const int32_t f0 = bid * F;
  const TileSpan sp = tile_span(a, f0, F);
  if (f0 >= sp.n_cols) return;          // the grid may be sized for a larger step
  const int32_t f_last = sp.f_last;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wm = wave % WM, wn = wave / WM;
  const int m = wm * 16 + lg * 4;       // the lane's channels m .. m + 3 (both convs)
  const bool m_ok = C == MT || m < C;   // (rows past C: padding)
  const bool pre_a = a.pa.pre_act != 0, pre_b = a.pre_act != 0;
  const float qs_a = PREC == 2 ? 1.0f / a.pa.act_scale : 1.0f;
  const float qs_b = PREC == 2 ? 1.0f / a.act_scale : 1.0f;
  const size_t r1 = (size_t)max(arow_cap * ROWB, F * XF * 4);
  unsigned char* wop_a = lds;                              // A's window rows, operand form
  float* xf = reinterpret_cast<float*>(lds);               // B's skip row of each column, FP32 (after A's MFMAs)
  unsigned char* wop_b = lds + r1;                         // B's window rows, operand form
  const float** rsrc = reinterpret_cast<const float**>(wop_b + (size_t)row_cap * ROWB);

  // A's weights (the wave's 16 rows, every chunk), both convs' biases and scales
  u4 alo[KCM], ahi[KCM];
  {
    const unsigned char* wrow = static_cast<const unsigned char*>(a.pa.W) + (int64_t)(wm * 16 + lr) * (Kpad * ES) + lg * 32;
#pragma unroll
    for (int c = 0; c < KCM; ++c) {
      alo[c] = *reinterpret_cast<const u4*>(wrow + c * 128);
      ahi[c] = *reinterpret_cast<const u4*>(wrow + c * 128 + 16);
    }
  }
  const f4 f4z = {0.f, 0.f, 0.f, 0.f}, f4o = {1.f, 1.f, 1.f, 1.f};
  const f4 bias_a = m_ok ? *reinterpret_cast<const f4*>(a.pa.B + m) : f4z;
  const f4 ws_a = PREC == 2 && m_ok ? *reinterpret_cast<const f4*>(a.pa.wscale + m) : f4o;
  const f4 bias_b = m_ok ? *reinterpret_cast<const f4*>(a.B + m) : f4z;
  const f4 ws_b = PREC == 2 && m_ok ? *reinterpret_cast<const f4*>(a.wscale + m) : f4o;
  // fused output conv: the lane's A operand of its per-tap sums (tap lr, channels m .. m + 3)
  f4 wa2 = f4z;
  if constexpr (FUSE) {
    if (lr < a.oc.k && m_ok) wa2 = *reinterpret_cast<const f4*>(a.oc.W + lr * C + m);
  }

  // ---- the streams of the tile: lane s of every wave forms stream s's
  // records; wave 0 publishes them ----
  const int e_first = sp.e0;
  const int n_seg = sp.n_seg;
  // the host sizes tiles so that these hold; never index LDS beyond them
  if (n_seg > kMaxStreams) return;
  int32_t n_rows = 0, n_acol = 0, n_arows = 0, n_cp = 0;
  {
    const Entry e = load_entry(a.ents + e_first + min(lane, n_seg - 1));
    WinSeg g{};
    PairSeg p{};
    int32_t ncol = 0, arows = 0, cpieces = 0;
    if (lane < n_seg) {
      g.cache = e.state + a.state_off + (int64_t)e.parity * a.state_len;
      g.mask_x = mask_lo(e, a.delay, a.out_num, a.out_den);
      g.mask_hi = mask_hi(e, a.delay, a.out_num, a.out_den);
      g.in_start = in_frames(a, e.off);
      g.out_start = out_frames(a, e.off);
      const int32_t T = out_frames(a, e.T);
      g.t_lo = lane == 0 ? f0 - g.out_start : 0;
      g.t_hi = lane == n_seg - 1 ? f_last - g.out_start : T - 1;
      g.r0 = g.t_lo;
      g.rows = g.t_hi - g.t_lo + 1 + LB;
      p.cache_a = e.state + a.pa.state_off + (int64_t)e.parity * a.pa.state_len;
      p.cache_b_next = e.state + a.state_off + (int64_t)(1 - e.parity) * a.state_len;
      p.mask_lo = mask_lo(e, a.pa.delay, a.out_num, a.out_den);
      p.mask_hi = mask_hi(e, a.pa.delay, a.out_num, a.out_den);
      p.in_start = g.in_start;
      p.T = T;
      // x1 frames of B's window: [max(0, t_lo - L_B), t_hi]; A's window rows: those plus L_A
      p.ta = max(0, g.t_lo - LB);
      ncol = g.t_hi - p.ta + 1;
      arows = ncol + LA;
      cpieces = max(0, min(LB - g.r0, g.rows)) * PPR;
    }
    // each stream's first B row, A column and A row: sums over the streams before it
    for (int s = 0; s < n_seg; ++s) {
      const int32_t r = __shfl(g.rows, s);
      const int32_t nc = __shfl(ncol, s);
      const int32_t ar = __shfl(arows, s);
      g.base += s < lane ? r : 0;
      p.acol0 += s < lane ? nc : 0;
      p.abase += s < lane ? ar : 0;
      n_rows += r;
      n_acol += nc;
      n_arows += ar;
      n_cp += __shfl(cpieces, s);
    }
    if (wave == 0 && lane < n_seg) {
      segs[lane] = g;
      psegs[lane] = p;
      if constexpr (FUSE) {
        WinSeg2 g2;
        g2.T = p.T;
        g2.cache2 = e.state + a.oc.state_off + (int64_t)e.parity * a.oc.state_len;
        g2.cache2_next = e.state + a.oc.state_off + (int64_t)(1 - e.parity) * a.oc.state_len;
        g2.out2 = e.out;
        g2.mask2_x = mask_lo(e, a.oc.delay, a.out_num, a.out_den);
        g2.mask2_hi = mask_hi(e, a.oc.delay, a.out_num, a.out_den);
        segs2[lane] = g2;
      }
    }
  }
  if (n_rows > row_cap || n_acol > NCOL || n_arows > arow_cap || n_cp > stash_cap || n_cp > CPRE * kThreads) return;
  __syncthreads();

  // ---- tables: B's columns, A's columns, A's window rows ----
  if (tid < F) {
    const int32_t f = f0 + tid;
    int s = 0;
    int8_t keep = -1;
    if (f <= f_last) {
      while (s + 1 < n_seg && segs[s + 1].out_start <= f) ++s;
      colbase[tid] = segs[s].base + (f - segs[s].out_start - segs[s].r0);
      const int64_t x = (int64_t)(f - segs[s].out_start) * a.out_den;
      keep = x < segs[s].mask_x || x >= segs[s].mask_hi ? 0 : 1;
    } else {
      colbase[tid] = 0;
      s = -1;
    }
    colkeep[tid] = keep;
    colseg[tid] = (int8_t)s;
  }
  for (int j = tid; j < NCOL; j += kThreads) {
    int32_t cb = 0, jb = 0, sl = -1;
    int8_t fl = 0;
    const float* sk = a.pa.B;              // a padding column reads a harmless row and is not used
    float* nx = nullptr;
    if (j < n_acol) {
      int s = 0;
      while (s + 1 < n_seg && psegs[s + 1].acol0 <= j) ++s;
      const PairSeg& p = psegs[s];
      const WinSeg& g = segs[s];
      const int32_t u = p.ta + (j - p.acol0);      // x1 frame of the stream
      cb = p.abase + (u - p.ta);                   // A's window row u (taps add dil_a rows)
      jb = g.base + (u + LB - g.r0);               // B's window row u + L_B
      const int32_t tt = u + LB - a.skip_off;      // the B frame whose skip row that is
      if (tt >= g.t_lo && tt <= g.t_hi) sl = g.out_start + tt - f0;
      const int64_t x = (int64_t)u * a.out_den;
      if (!(x < p.mask_lo || x >= p.mask_hi)) fl |= 1;
      const int32_t r = u + a.pa.skip_off;         // A's skip: its window row u + skip_off
      sk = r < LA ? p.cache_a + (int64_t)r * C : a.pa.in_buf + ((int64_t)p.in_start + r - LA) * C;
      if (u >= p.T - LB && u >= g.t_lo && u <= g.t_hi) {
        fl |= 2;
        nx = p.cache_b_next + (int64_t)(u - (p.T - LB)) * C;
      }
    }
    acb[j] = cb;
    ajb[j] = jb;
    aslot[j] = (int16_t)sl;
    aflag[j] = fl;
    askip[j] = sk;
    anext[j] = nx;
  }
  for (int j = tid; j < n_arows; j += kThreads) {
    int s = 0;
    while (s + 1 < n_seg && psegs[s + 1].abase <= j) ++s;
    const PairSeg& p = psegs[s];
    const int32_t r = p.ta + (j - p.abase);        // A's window row
    rsrc[j] = r < LA ? p.cache_a + (int64_t)r * C : a.pa.in_buf + ((int64_t)p.in_start + r - LA) * C;
  }
  __syncthreads();

  // ---- loads: B's cache rows, A's skip values of the lane's columns, A's
  // window rows (operand form) ----
  // (B's cache rows stay in registers until region 1 is free)
  // cdst: the piece's operand offset (C ch + row) in the low 16 bits, its
  // skip-row offset (XF slot + ch, 0x7fff: none) in the high 15; -1: no piece
  f4 cpre[CPRE];
  int32_t cdst[CPRE];
#pragma unroll
  for (int p = 0; p < CPRE; ++p) {
    cdst[p] = -1;
    cpre[p] = f4{0.f, 0.f, 0.f, 0.f};
    int32_t idx = tid + p * kThreads;
    for (int s = 0; s < n_seg; ++s) {
      const WinSeg& g = segs[s];
      const int32_t n = max(0, min(LB - g.r0, g.rows)) * PPR;
      if (idx < n) {
        const int32_t i = idx / PPR;
        const int ch = (idx - i * PPR) * 4;
        cpre[p] = gload<f4>(g.cache + (int64_t)(g.r0 + i) * C + ch);
        const int32_t tt = g.r0 + i - a.skip_off;   // the B frame whose skip row this is
        const int32_t sk = tt >= g.t_lo && tt <= g.t_hi ? (g.out_start + tt - f0) * XF + ch : 0x7fff;
        cdst[p] = ((g.base + i) * C + ch) | sk << 16;
        break;
      }
      idx -= n;
    }
  }
  f4 skv[NCW];
#pragma unroll
  for (int i = 0; i < NCW; ++i) skv[i] = m_ok ? gload<f4>(askip[(wn * NCW + i) * 16 + lr] + m) : f4z;
  {
    const int32_t n_pieces = n_arows * PPR;
    for (int32_t i0 = 0; i0 < n_pieces; i0 += kThreads * SB) {
      f4 v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int32_t idx = i0 + u * kThreads + tid;
        v[u] = f4{0.f, 0.f, 0.f, 0.f};
        if (idx < n_pieces) v[u] = gload<f4>(rsrc[idx / PPR] + (idx % PPR) * 4);
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int32_t idx = i0 + u * kThreads + tid;
        if (idx >= n_pieces) continue;
        unsigned char* dst = wop_a + (idx / PPR) * ROWB + (idx % PPR) * 4 * ES;
        store_operand<PREC>(dst, v[u], pre_a, qs_a);
      }
    }
  }
  __syncthreads();

  // ---- A: the wave's 16 rows x its A column blocks (column blocks
  // wn * NCW .. + NCW - 1) ----
  const int ncba = (n_acol + 15) / 16;
  const int nc0 = wn * NCW;
  f4 aacc[NCW];
  {
    int cb[NCW];
#pragma unroll
    for (int i = 0; i < NCW; ++i) {
      cb[i] = acb[(nc0 + i) * 16 + lr] * ROWB;
      aacc[i] = f4{0.f, 0.f, 0.f, 0.f};
    }
    // two groups of column blocks, each over every chunk (a column's chain of
    // MFMAs is the same; half the operand registers)
    constexpr int G = NCW / 2;
#pragma unroll
    for (int g0 = 0; g0 < NCW; g0 += G) {
      if (nc0 + g0 >= ncba) break;
#pragma unroll
      for (int c = 0; c < KCM; ++c) {
        u4 blo[G], bhi[G];
        win_chunk_reads<ES, G, C, KX>(a.fd_cin, a.pa.dil, c, lg, Kreal, C, ROWB, wop_a, cb + g0, blo, bhi);
#pragma unroll
        for (int q = 0; q < G; ++q)
          if (nc0 + g0 + q < ncba) aacc[g0 + q] = mfma32<PREC>(alo[c], ahi[c], blo[q], bhi[q], aacc[g0 + q]);
      }
    }
  }
  // B's weights (their latency hides behind x1's epilogue)
  u4 blw[KCM], bhw[KCM];
  {
    const unsigned char* wrow = static_cast<const unsigned char*>(a.W) + (int64_t)(wm * 16 + lr) * (Kpad * ES) + lg * 32;
#pragma unroll
    for (int c = 0; c < KCM; ++c) {
      blw[c] = *reinterpret_cast<const u4*>(wrow + c * 128);
      bhw[c] = *reinterpret_cast<const u4*>(wrow + c * 128 + 16);
    }
  }
  __syncthreads();   // every wave is past A's operand rows: region 1 takes B's FP32 rows

  // ---- x1: A's epilogue, B's window rows (FP32 and operand), B's next cache ----
  int32_t jbs[NCW], sls[NCW];
  int fls[NCW];
#pragma unroll
  for (int i = 0; i < NCW; ++i) {        // every column's record first: one wait
    jbs[i] = ajb[(nc0 + i) * 16 + lr];
    sls[i] = aslot[(nc0 + i) * 16 + lr];
    fls[i] = aflag[(nc0 + i) * 16 + lr];
  }
#pragma unroll
  for (int i = 0; i < NCW; ++i) {
    const int col = (nc0 + i) * 16 + lr;
    if (nc0 + i >= ncba || col >= n_acol || !m_ok) continue;
    const int32_t jb = jbs[i];
    const int fl = fls[i];
    f4 v = aacc[i];
    if (PREC == 2) v = v * (ws_a * a.pa.act_scale);
    v = v + bias_a;
    v = v + skv[i];
    if (!(fl & 1)) v = f4{0.f, 0.f, 0.f, 0.f};
    if (sls[i] >= 0) *reinterpret_cast<f4*>(xf + (size_t)sls[i] * XF + m) = v;
    store_operand<PREC>(wop_b + (size_t)jb * ROWB + m * ES, v, pre_b, qs_b);
    if (fl & 2) gstore<f4>(anext[col] + m, v);
  }
  // B's window rows from its cache (rows below L_B)
#pragma unroll
  for (int p = 0; p < CPRE; ++p) {
    if (cdst[p] < 0) continue;
    const f4 v = cpre[p];
    const int32_t od = cdst[p] & 0xffff, sk = cdst[p] >> 16;
    const int32_t jr = od / C;
    const int ch = od - jr * C;
    if (sk != 0x7fff) *reinterpret_cast<f4*>(xf + sk) = v;
    store_operand<PREC>(wop_b + (size_t)jr * ROWB + ch * ES, v, pre_b, qs_b);
  }
  __syncthreads();

  // ---- B: operands from its staged rows, the skip from its FP32 rows ----
  int cbb[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) cbb[nb] = colbase[wn * (F / WN) + nb * 16 + lr] * ROWB;
  f4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < KCM; ++c) {
    u4 blo[NB], bhi[NB];
    win_chunk_reads<ES, NB, C, KX>(a.fd_cin, a.dil, c, lg, Kreal, C, ROWB, wop_b, cbb, blo, bhi);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma32<PREC>(blw[c], bhw[c], blo[nb], bhi[nb], acc[nb]);
  }
  if constexpr (FUSE) {
    // the output conv in the epilogue; its per-tap scratch takes B's operand rows
    fused_out_epilogue<PREC, MT, NB, F>(
        a, acc, m, bias_b, ws_b, f0, [&](int col) { return xf + (size_t)col * XF; }, segs,
        segs2, colseg, n_seg, wa2, wop_b);
    return;
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = wn * (F / WN) + nb * 16 + lr;
    const int keep = colkeep[col];
    if (keep < 0 || !m_ok) continue;
    const int32_t f = f0 + col;
    f4 v = acc[nb];
    if (PREC == 2) v = v * (ws_b * a.act_scale);
    v = v + bias_b;
    if (a.residual) v = v + *reinterpret_cast<const f4*>(xf + (size_t)col * XF + m);
    if (!keep) v = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t o = (int64_t)f * a.cout + m;
    if (!a.twin_only) gstore<f4>(a.out_buf + o, v);
    if (a.out_twin) store_twin(a, o, v);
  }
}

int w_esize(int prec) { return prec == 0 ? 4 : (prec == 1 ? 2 : 1); }
int w_kchunk(int prec) { return prec == 0 ? 32 : (prec == 1 ? 64 : 128); }

// Tile shape: the gather kernel's M tile (the packed weights are padded to
// it); 64 frames per wave for inputs of up to 64 channels, 32 for 128.
int win_mt(int cout) { return cout <= 32 ? 32 : 64; }
int win_nb(int cin) { return cin <= 64 ? 4 : 2; }
int win_f(int mt, int nb) { return nb * 16 * (4 / (mt / 16)); }
// K chunks the kernel holds in registers
int win_kcm(int prec, int cin) {
  if (prec == 0) return cin <= 32 ? 3 : 6;
  return cin <= 64 ? (prec == 1 ? 3 : 2) : (prec == 1 ? 6 : 3);
}
// operand rows plus the skip rows (allocated whether or not the layer has a skip)
// operand rows, skip rows, then per staged row its source (8 B) and skip slot (4 B)
int64_t win_lds_bytes(int64_t rows, int cin, int prec, int F) {
  return rows * (cin * w_esize(prec) + 16) + (int64_t)F * (cin + 4) * 4 + rows * 12;
}

// The frames of a fused output conv that its window tiles leave (see
// out_tail_frame).  Blocks [0, bnd_blocks): one lane per frame f0 + i, i < L,
// after every tile start f0 but the first, P of its rows (all of this step)
// from out_buf.  Blocks after: one wave per stream of the step, which forms P
// of the stream's L cache rows (one MFMA column each, L <= 16) and finishes
// its first L frames.
template <int CIN>
__global__ void __launch_bounds__(kThreads) conv_out_tail_kernel(LayerArgs a, int32_t tile_frames, int32_t n_bnd,
                                                                 int32_t bnd_blocks) {
  __shared__ __attribute__((aligned(16))) float pc[kThreads / 64][16][kOutTaps];
  const float* W = static_cast<const float*>(a.W);   // [k][cin]
  if ((int32_t)blockIdx.x < bnd_blocks) {
    const int32_t idx = (int32_t)blockIdx.x * kThreads + (int32_t)threadIdx.x;
    if (idx >= n_bnd) return;
    const int32_t b = idx / a.L;
    const int32_t f0 = (b + 1) * tile_frames;
    const int32_t f = f0 + (idx - b * a.L);
    if (f >= step_out(a)) return;   // the grid may be sized for a larger step
    // P of the frame's rows f - L .. f (all inside this step: f0 >= 2 L) are
    // read together with the frame's stream record
    float p[kOutTaps];
#pragma unroll
    for (int kk = 0; kk < kOutTaps; ++kk)
      p[kk] = kk < a.k ? gload<float>(a.in_buf + (int64_t)(f - a.L + a.dil * kk) * CIN + kk) : 0.f;
    const Entry e = load_entry(a.ents + entry_of_out(a, f));
    const int32_t out_start = out_frames(a, e.off);
    const int32_t t = f - out_start;
    if (!(out_start < f0 && f - a.L < f0) || t < a.L) return;   // its tile's, or a stream start
    float o = a.B[0];
#pragma unroll
    for (int kk = 0; kk < kOutTaps; ++kk)
      if (kk < a.k) o = o + p[kk];
    if (a.post_act == 2) o = tanhf(o);
    if (masked(a, e, t)) o = 0.f;
    gstore<float>(e.out + t, o);
    return;
  }
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int32_t ei = ((int32_t)blockIdx.x - bnd_blocks) * (kThreads / 64) + wave;
  const bool live = ei < step_ents(a);   // uniform in the wave
  const bool pre = a.pre_act != 0;
  const Entry e = load_entry(a.ents + (live ? ei : 0));
  // lane t < L finishes the stream's frame t: P of its rows past the cache
  // (the stream's first frames, from out_buf) are read before the cache rows'
  // P are formed
  const int32_t t = lane;
  const bool fin = live && t < a.L && t < out_frames(a, e.T);
  const int32_t out_start = out_frames(a, e.off);
  float q[kOutTaps];
#pragma unroll
  for (int kk = 0; kk < kOutTaps; ++kk) {
    const int w = t + a.dil * kk;   // row of [cache | new frames]
    q[kk] = fin && kk < a.k && w >= a.L ? gload<float>(a.in_buf + (int64_t)(out_start + w - a.L) * CIN + kk) : 0.f;
  }
  if (live) {
    const float* cache = e.state + a.state_off + (int64_t)e.parity * a.state_len;
    f4 P = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < CIN / 16; ++g) {
      const int c = g * 16 + lg * 4;
      const f4 wa = lr < a.k ? *reinterpret_cast<const f4*>(W + lr * CIN + c) : f4{0.f, 0.f, 0.f, 0.f};
      f4 y = lr < a.L ? gload<f4>(cache + (int64_t)lr * CIN + c) : f4{0.f, 0.f, 0.f, 0.f};
      y = f4{act(y.x, pre), act(y.y, pre), act(y.z, pre), act(y.w, pre)};
      const f4 d = tap_mfma(wa, y);
      P = g == 0 ? d : P + d;
    }
    if (lg < kOutTaps / 4) *reinterpret_cast<f4*>(&pc[wave][lr][lg * 4]) = P;   // [cache row][tap]
  }
  __syncthreads();
  if (!fin) return;
  float o = a.B[0];
#pragma unroll
  for (int kk = 0; kk < kOutTaps; ++kk) {
    if (kk < a.k) {
      const int w = t + a.dil * kk;
      o = o + (w < a.L ? pc[wave][w][kk] : q[kk]);
    }
  }
  if (a.post_act == 2) o = tanhf(o);
  if (masked(a, e, t)) o = 0.f;
  gstore<float>(e.out + t, o);
}

}  // namespace

int32_t conv_win_tile_frames(int cin, int cout) { return win_f(win_mt(cout), win_nb(cin)); }

bool conv_win_out_fusable(int cin, int cout, int k, int dil) {
  // all output channels in one M tile (the tail launch has instances for 32,
  // 48 and 64), a tile shape with fused variants, and the taps of a boundary
  // frame reaching no further than the previous tile
  if ((cout != 32 && cout != 48 && cout != 64) || win_nb(cin) != 4 || k < 1 || k > kOutTaps || dil < 1) return false;
  const int L = dil * (k - 1);
  return L <= 16 && 2 * L <= conv_win_tile_frames(cin, cout);   // the tail forms P of <= 16 cache rows
}

hipError_t launch_conv_out_tail(const LayerArgs& a, int32_t tile_frames, hipStream_t s) {
  if (a.L <= 0 || tile_frames <= 0 || a.cin % 4 != 0) return a.L <= 0 ? hipSuccess : hipErrorInvalidValue;
  const int64_t n_tiles = (a.n_out + tile_frames - 1) / tile_frames;
  const int64_t n_bnd = std::max<int64_t>(n_tiles - 1, 0) * a.L;
  const int64_t bnd_blocks = (n_bnd + kThreads - 1) / kThreads;
  const int64_t blocks = bnd_blocks + ((int64_t)a.n_ent + kThreads / 64 - 1) / (kThreads / 64);
  if (blocks == 0) return hipSuccess;
#define SC_TAIL(C)                                                                                         \
  hipLaunchKernelGGL((conv_out_tail_kernel<C>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a, tile_frames, \
                     (int32_t)n_bnd, (int32_t)bnd_blocks)
  if (a.cin == 32) SC_TAIL(32);
  else if (a.cin == 48) SC_TAIL(48);
  else if (a.cin == 64) SC_TAIL(64);
  else return hipErrorInvalidValue;
#undef SC_TAIL
  return hipGetLastError();
}

int32_t conv_win_rows(int cin, int cout, int k, int dil, int stride, int L, int64_t min_frames, int prec) {
  if (stride != 1 || !conv_mfma_supported(cin, cout, k, stride, prec)) return 0;
  // up to 64 input channels: measured slower than the gathering kernel at 128
  // (32-frame tiles re-stage too large a halo per output)
  if (cin > 64 || cin % 16 != 0 || cout % 16 != 0 || min_frames < 1) return 0;
  if (L != dil * (k - 1)) return 0;
  const int kc = w_kchunk(prec);
  const int Kpad = (k * cin + kc - 1) / kc * kc;
  if (Kpad * w_esize(prec) / 128 > win_kcm(prec, cin)) return 0;
  const int mt = win_mt(cout);
  if (win_nb(cin) == 2 && mt != 64) return 0;
  const int F = win_f(mt, win_nb(cin));
  const int64_t max_seg = (F - 1 + min_frames - 1) / min_frames + 1;   // streams one tile may touch
  if (max_seg > kMaxStreams) return 0;
  const int64_t rows = F + (int64_t)L * max_seg;
  if (win_lds_bytes(rows, cin, prec, F) > 64 * 1024) return 0;
  return (int32_t)rows;
}

hipError_t launch_conv_win(const LayerArgs& a, int prec, int32_t row_cap, hipStream_t s) {
  const int MT = win_mt(a.cout);
  const int NB = win_nb(a.cin);
  const int F = win_f(MT, NB);
  const int KCM = win_kcm(prec, a.cin);
  const int n_mt = (a.cout + MT - 1) / MT;
  const int64_t n_nt = (a.n_out + F - 1) / F;
  const int kc = w_kchunk(prec);
  const int Kreal = a.k * a.cin;
  const int Kpad = (Kreal + kc - 1) / kc * kc;
  const int64_t items = (int64_t)a.n_ent * a.L * a.cin / 4;   // 4 channels per cache-update item
  const int extra = (int)std::min<int64_t>((items + kThreads - 1) / kThreads, 1024);
  const int64_t grid = (int64_t)n_mt * n_nt + extra;
  if (grid <= 0) return hipSuccess;
  const bool fuse = a.oc.k > 0;
  if (fuse && (a.cout > MT || a.cout % 16 != 0 || NB != 4 || !a.out_buf)) return hipErrorInvalidValue;
  size_t lds = (size_t)win_lds_bytes(row_cap, a.cin, prec, F);
  // per-wave partial tap sums of the output conv
  if (fuse) lds = std::max(lds, (size_t)(MT / 16) * F * kOutTaps * 4);
  const FastDiv fd_per_ent = make_fastdiv((uint32_t)std::max(a.L * a.cin / 4, 1));
  const FastDiv fd_ppr = make_fastdiv((uint32_t)(a.cin / 4));   // 16-byte pieces per staged row
  // an instance for cin == MT where one exists (with kx: K fills the chunks)
  const int cin_t = a.cin == MT ? MT : 0;
  const bool kx = cin_t > 0 && Kreal == Kpad && Kpad * w_esize(prec) == KCM * 128;
#define SC_WINC(P, M, N, K, FU, CI, X)                                                                     \
  if (prec == P && MT == M && NB == N && KCM == K && fuse == FU && cin_t == CI && kx == X) {              \
    hipLaunchKernelGGL((conv_win_kernel<P, M, N, K, FU, CI, X>), dim3((unsigned)grid), dim3(kThreads), lds, s, a, \
                       n_mt, (int)n_nt, Kpad, Kreal, row_cap, extra, fd_per_ent, fd_ppr);                  \
    return hipGetLastError();                                                                              \
  }
  SC_WINC(1, 32, 4, 3, false, 32, false) SC_WINC(1, 32, 4, 3, true, 32, false)
  SC_WINC(1, 64, 4, 3, false, 64, true) SC_WINC(1, 64, 4, 3, true, 64, true)
  SC_WINC(2, 32, 4, 2, false, 32, false) SC_WINC(2, 32, 4, 2, true, 32, false)
  SC_WINC(2, 64, 4, 2, false, 64, false) SC_WINC(2, 64, 4, 2, true, 64, false)
#undef SC_WINC
#define SC_WIN(P, M, N, K, FU)                                                                              \
  if (prec == P && MT == M && NB == N && KCM == K && fuse == FU) {                                         \
    hipLaunchKernelGGL((conv_win_kernel<P, M, N, K, FU>), dim3((unsigned)grid), dim3(kThreads), lds, s, a, \
                       n_mt, (int)n_nt, Kpad, Kreal, row_cap, extra, fd_per_ent, fd_ppr);                  \
    return hipGetLastError();                                                                              \
  }
  SC_WIN(0, 32, 4, 3, false) SC_WIN(0, 64, 4, 3, false) SC_WIN(0, 64, 4, 6, false)
  SC_WIN(1, 32, 4, 3, false) SC_WIN(1, 64, 4, 3, false) SC_WIN(1, 64, 2, 6, false)
  SC_WIN(2, 32, 4, 2, false) SC_WIN(2, 64, 4, 2, false) SC_WIN(2, 64, 2, 3, false)
  SC_WIN(0, 32, 4, 3, true) SC_WIN(0, 64, 4, 3, true) SC_WIN(0, 64, 4, 6, true)
  SC_WIN(1, 32, 4, 3, true) SC_WIN(1, 64, 4, 3, true)
  SC_WIN(2, 32, 4, 2, true) SC_WIN(2, 64, 4, 2, true)
#undef SC_WIN
  return hipErrorInvalidValue;
}

namespace {
// the instances of the fused kernel: (precision, M tile, transposed-conv K
// chunks, M blocks per wave) -> the column blocks a tile may need.  Only the
// 32-row tile: its 128-frame tiles amortise the transposed conv's weights
// (r * 32 rows) over enough frames; a 64-row tile covers 64 frames and
// reloads r * 64 weight rows per tile, which measured slower than the two
// launches.
int ct_col_blocks(int prec, int mt, int kct, int mbw) {
  if (mt == 32 && mbw == 1 && ((prec == 1 && kct == 2) || (prec == 2 && kct == 2))) return 6;
  return 0;
}
// staged input rows of kct * 64 bytes (+16), overlaid by the FP32 window
// rows, then the operand rows
int64_t ct_lds_bytes(int64_t rows, int64_t xrows, int64_t stash, int mt, int prec, int kct) {
  return std::max(xrows * (kct * 64 + 16), rows * mt * 4) + stash * 16 + rows * (mt * w_esize(prec) + 16);
}
}  // namespace

int32_t convt_win_rows(int cin, int cout, int k, int dil, int L, int r, int ct_cin, int prec, int64_t min_frames,
                       int32_t* xrow_cap, int32_t* stash_cap) {
  *xrow_cap = 0;
  *stash_cap = 0;
  // the transposed conv's input frames are staged in 16-byte pieces
  if (prec < 1 || prec > 2 || r < 1 || ct_cin < 1 || ct_cin % (16 / w_esize(prec)) != 0) return 0;
  const int32_t rows = conv_win_rows(cin, cout, k, dil, 1, L, min_frames, prec);
  const int MT = win_mt(cout);
  // one M tile, a residual conv (cin == cout), and every stream bringing at
  // least L frames (the tiles write the whole next cache)
  if (rows <= 0 || cout != MT || cin != cout || win_nb(cin) != 4 || min_frames < L || (r * MT) % 64 != 0) return 0;
  const int kc = w_kchunk(prec);
  const int half = (ct_cin + kc - 1) / kc * kc;
  const int kct = 2 * half * w_esize(prec) / 128;
  const int ncb = ct_col_blocks(prec, MT, kct, r * MT / 64);
  if (ncb == 0) return 0;
  const int F = win_f(MT, 4);
  const int64_t max_seg = (F - 1 + min_frames - 1) / min_frames + 1;
  // per stream: its x frames (its own plus L before) over r, two partial
  // columns at the ends, and the carry column; one staged input row more
  // than columns per stream; the window's cache rows fit two f4 per thread
  const int64_t cols = (F + (int64_t)L * max_seg + r - 1) / r + 3 * max_seg;
  const int64_t xrows = (cols + max_seg + 15) / 16 * 16;
  const int64_t stash = max_seg * L * (MT / 4);
  const int kc_conv = w_kchunk(prec);
  const int kcm = (k * cin + kc_conv - 1) / kc_conv * kc_conv * w_esize(prec) / 128;
  if (cols > ncb * 16 || stash > 2 * 256 || ct_lds_bytes(rows, xrows, stash, MT, prec, kct) > 64 * 1024 ||
      kcm != (prec == 1 ? 2 : 1))
    return 0;
  *xrow_cap = (int32_t)xrows;
  *stash_cap = (int32_t)stash;
  return rows;
}

hipError_t launch_convt_win(const LayerArgs& a, int prec, int32_t row_cap, int32_t xrow_cap, int32_t stash_cap,
                            hipStream_t s) {
  const int MT = win_mt(a.cout);
  const int NB = win_nb(a.cin);
  const int F = win_f(MT, NB);
  const int kc = w_kchunk(prec);
  const int Kreal = a.k * a.cin;
  const int Kpad = (Kreal + kc - 1) / kc * kc;
  const int KCM = Kpad * w_esize(prec) / 128;
  const int kct = a.ct.Kpad * w_esize(prec) / 128;
  const int mbw = a.ct.r * MT / 64;
  if (a.cout != MT || NB != 4 || a.ct.r <= 0 || a.ct.r * MT != 64 * mbw || kct % 2 != 0 ||
      a.fd_cin.d != (uint32_t)a.cin || !a.out_buf || ct_col_blocks(prec, MT, kct, mbw) == 0)
    return hipErrorInvalidValue;
  const int64_t n_nt = (a.n_out + F - 1) / F;
  if (n_nt <= 0) return hipSuccess;
  const size_t lds = (size_t)ct_lds_bytes(row_cap, xrow_cap, stash_cap, MT, prec, kct);
#define SC_CTWIN(P, M, K, KT, MB, NCB)                                                                      \
  if (prec == P && MT == M && KCM == K && kct == KT && mbw == MB) {                                        \
    hipLaunchKernelGGL((convt_win_kernel<P, M, 4, K, KT, MB, NCB>), dim3((unsigned)n_nt), dim3(kThreads), lds, \
                       s, a, (int)n_nt, Kpad, Kreal, row_cap, xrow_cap, stash_cap);                                     \
    return hipGetLastError();                                                                              \
  }
  SC_CTWIN(1, 32, 2, 2, 1, 6) SC_CTWIN(2, 32, 1, 2, 1, 6)
#undef SC_CTWIN
  return hipErrorInvalidValue;
}


namespace {
// x1 frames a pair tile computes at most (A column blocks x 16), by channels
int pair_cols(int c) { return c == 32 ? 192 : 96; }
// A's window rows in operand form, overlaid by B's skip rows in FP32 (one per
// tile column, row stride c + 4); B's window rows in operand form and A's row
// sources, overlaid by the fused output conv's per-tap scratch
int64_t pair_lds_bytes(int c, int64_t rows, int64_t arows, int prec, bool fuse) {
  const int64_t rowb = c * w_esize(prec) + 16;
  const int mt = win_mt(c);
  const int64_t F = win_f(mt, 4);
  const int64_t scratch = fuse ? (int64_t)(mt / 16) * kOutTaps * F * 4 : 0;
  return std::max(arows * rowb, F * (c + 4) * 4) + std::max(rows * rowb + arows * 8, scratch);
}
int pair_kchunks(int c, int k, int prec) {
  const int kc = w_kchunk(prec);
  return (k * c + kc - 1) / kc * kc * w_esize(prec) / 128;
}
}  // namespace

int32_t conv_pair_rows(int c, int k, int dil_a, int dil_b, int prec, int64_t min_frames, bool fuse,
                       int32_t* arow_cap, int32_t* stash_cap) {
  *arow_cap = 0;
  *stash_cap = 0;
  // instances: 64 channels (no fused output conv), 48 (on a 64-row tile) and
  // 32 channels (with or without)
  if ((c != 64 && c != 48 && c != 32) || (c == 64 && fuse) || k != 3 || prec < 1 || prec > 2 || dil_a < 1 ||
      dil_b < 1 || min_frames < 1)
    return 0;
  const int LA = dil_a * (k - 1), LB = dil_b * (k - 1);
  // every stream brings at least L_B frames: B's next cache comes from x1 alone
  if (min_frames < LB) return 0;
  const int F = win_f(win_mt(c), 4);
  const int64_t max_seg = (F - 1 + min_frames - 1) / min_frames + 1;   // streams one tile may touch
  if (max_seg > kMaxStreams) return 0;
  const int64_t rows = F + (int64_t)LB * max_seg;     // B's window rows
  const int64_t acols = F + (int64_t)LB * max_seg;    // x1 frames computed
  const int64_t arows = acols + (int64_t)LA * max_seg;
  const int64_t stash = (int64_t)LB * max_seg * (c / 4);
  if (acols > pair_cols(c) || stash > 2 * kThreads || pair_lds_bytes(c, rows, arows, prec, fuse) > 64 * 1024)
    return 0;
  *arow_cap = (int32_t)arows;
  *stash_cap = (int32_t)stash;
  return (int32_t)rows;
}

hipError_t launch_conv_pair(const LayerArgs& a, int prec, int32_t row_cap, int32_t arow_cap, int32_t stash_cap,
                            hipStream_t s) {
  const int C = a.cout;
  const bool fuse = a.oc.k > 0;
  const int F = win_f(win_mt(C), 4);
  const int kc = w_kchunk(prec);
  const int Kreal = a.k * C;
  const int Kpad = (Kreal + kc - 1) / kc * kc;
  const int KCM = pair_kchunks(C, a.k, prec);
  if ((C != 64 && C != 48 && C != 32) || a.cin != C || a.k != 3 || a.pa.L != a.pa.dil * 2 || a.L != a.dil * 2 ||
      !a.out_buf || a.fd_cin.d != (uint32_t)C || (fuse && (C == 64 || a.oc.k > kOutTaps)))
    return hipErrorInvalidValue;
  const int64_t n_nt = (a.n_out + F - 1) / F;
  const int64_t items = (int64_t)a.n_ent * a.pa.L * C / 4;   // 4 channels per cache-update item
  const int extra = (int)std::min<int64_t>((items + kThreads - 1) / kThreads, 1024);
  const int64_t grid = n_nt + extra;
  if (grid <= 0) return hipSuccess;
  const size_t lds = (size_t)pair_lds_bytes(C, row_cap, arow_cap, prec, fuse);
  const FastDiv fd_per_ent = make_fastdiv((uint32_t)std::max(a.pa.L * C / 4, 1));
#define SC_PAIR(P, M, K, NC, FU, CHN)                                                                      \
  if (prec == P && C == CHN && KCM == K && fuse == FU) {                                                   \
    hipLaunchKernelGGL((conv_pair_kernel<P, M, 4, K, NC, FU, CHN>), dim3((unsigned)grid), dim3(kThreads), lds, s, \
                       a, (int)n_nt, Kpad, Kreal, row_cap, arow_cap, stash_cap, extra, fd_per_ent);         \
    return hipGetLastError();                                                                              \
  }
  SC_PAIR(1, 64, 3, 6, false, 64) SC_PAIR(2, 64, 2, 6, false, 64)
  SC_PAIR(1, 64, 3, 6, false, 48) SC_PAIR(1, 64, 3, 6, true, 48) SC_PAIR(2, 64, 2, 6, false, 48)
  SC_PAIR(2, 64, 2, 6, true, 48)
  SC_PAIR(1, 32, 2, 12, false, 32) SC_PAIR(1, 32, 2, 12, true, 32) SC_PAIR(2, 32, 1, 12, false, 32)
  SC_PAIR(2, 32, 1, 12, true, 32)
#undef SC_PAIR
  return hipErrorInvalidValue;
}

}  // namespace sc
