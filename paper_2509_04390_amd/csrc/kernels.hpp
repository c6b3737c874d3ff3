// kernels.hpp -- gfx950 kernels of the partitioned convolution.
//
// One launch per audio block.
//
// The frequency-domain delay line (Sec. IV step 2) gives every output block
//     Y_l[k] = sum_q sum_{p<K} H_{l,q,p}[k] * X_q[(n - p) mod K][k].
// Only the p = 0 term needs the block that has just arrived, and the p = 1
// term needs the previous block's spectrum; every term p >= 2 uses spectra
// that were in the delay line one block earlier.  Launch n of k_block
// therefore runs two kinds of workgroups side by side (three with
// non-uniform partitions, whose later tiers add transform workgroups, see
// "Later tiers" below):
//
//   head workgroups (one per output, dispatched first, latency critical):
//   real FFT of each input's window [x_{n-1}, x_n] (Sec. IV step
//   1, batched in LDS), store it into ring slot n mod K, add
//   sum_q H_{l,q,0} X_q(n) + H_{l,q,1} X_q(n-1) to the partial sums of the
//   terms p >= 2 that the previous launch prepared, inverse real FFT, keep
//   the second half of the 2B samples (overlap-save, Sec. IV step 3), write
//   the output block; the last head workgroup then raises a host-visible
//   completion flag;
//
//   tail workgroups (bandwidth bound): work item i covers a group of G
//   outputs, one input, a partition range [p0, p1) with p0 >= 2 and a slice
//   of bins, and writes sum_{p in [p0,p1)} H_{l,q,p} X_q[(n+1-p) mod K] for
//   the NEXT block into its partial-sum slot.
//
// Partial sums are double-buffered by block parity: launch n reads parity
// n & 1 (heads) and writes parity (n+1) & 1 (tails).  The tails read ring
// slots n-1 ... n+2-K, never slot n, which the heads write in the same
// launch.  Each slot is written by exactly one item and read in a fixed
// order, so results are reproducible bit for bit; the sum is the same as
// forming all K terms at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace rta {

constexpr int kThreads = 256;
constexpr int kMaxTiers = 8;
constexpr int kUnroll = 4;  // rows in flight per lane, FP32 spectra (16-byte loads)
#ifndef RTA_UNROLL16
#define RTA_UNROLL16 4
#endif
constexpr int kUnroll16 = RTA_UNROLL16;  // rows in flight per lane, 16-bit spectra (8-byte loads)

enum ItemKind : int32_t {
  K_MAC = 0,    // tail: multiply-accumulate of a partition range
  K_NOP = 1,    // padding
  // later tiers: each 2P_t-point real transform is split into a column pass
  // and a row pass (P_t = N1 N2 complex points), run by several small
  // workgroups in consecutive launches
  K_FFT_A = 2,  // input frame -> N2-point transforms of its columns
  K_FFT_B = 3,  // N1-point transforms of column pairs -> packed spectrum -> ring
  K_FIN_A = 4,  // partial sums of column pairs -> N1-point inverse transforms
  K_FIN_B = 5   // N2-point inverse transforms of rows -> output ring
};

struct Item {          // one workgroup's work in one block (96 bytes)
  int32_t kind;        // ItemKind
  int32_t w;           // K_MAC: bins of the slice (divides P; W/C lanes per row);
                       // tier passes: columns (rows) or column pairs per item
  int32_t tier;
  int32_t group;       // reduction group (outputs l0 .. l0+nl-1)
  int32_t q;           // input channel; K_FIN_*: output within the group
  int32_t p0, p1;      // partition range
  int32_t k0;          // K_MAC: first bin of the slice; tier passes: index of
                       // the item within its pass
  int32_t slot;        // partial-sum slot (tier-local)
  int32_t acc;         // K_MAC of a later tier: add to the slot (0: store)
  int32_t lag;         // tiers >= 1: launch index minus the block in which
                       // the frame's input completed
  int32_t nl;          // K_MAC: outputs of its group
  // K_MAC, per output g of the group: the end of the partitions to read,
  // min(p1, partitions of pair (l0 + g, q)) (0: no path), and that pair's
  // first spectrum row.  Carried here so that a tail workgroup needs one
  // load (its item) before it streams, not a chain of table lookups.
  int32_t pend[4];
  int64_t row[4];
};
static_assert(sizeof(Item) == 96, "Item layout");

struct Group {         // outputs reduced together (16 bytes)
  int32_t l0, nl;      // first output, outputs in the group (<= G)
  int32_t slot0, nslot;
};

struct DevTier {
  const void* H;             // spectra rows [row][P] of the storage type
  const int64_t* pair_row;   // [L*Q] first row of pair (l,q), -1 = no path
  const int32_t* pair_K;     // [L*Q] partitions of pair (l,q)
  float2* X;                 // FDL ring [Q][K][P]
  float2* partial;           // [2][slots][G][P], by block parity
  const float2* tw;          // W_P^j (j<P) then W_2P^k (k<P)
  float* oring;              // tiers >= 1: output ring [L][R]
  float2* tfwd;              // tiers >= 1: forward column-pass results [Q][P]
  float2* tinv;              // tiers >= 1: inverse column-pass results [L][P]
  int64_t offset;            // first filter tap of the tier (o_t)
  int32_t P, logP, K, nslots;
  int32_t r;                 // P / B: blocks per frame
  int32_t lg1;               // tiers >= 1: log2 N1, P = N1 N2, N1 <= N2
  int32_t r3;                // 1: P = 3 * 2^logP (the n_f = 3 n_x first tier:
                             // B-tap partitions, 3B-point transforms, 3B/2 bins)
  int32_t pad5;
};

// Feedback convolution fused into the synthesis launch (Sec. III-A Eq. 3,
// Sec. V).  Its inputs are the synthesis outputs y_l, its outputs the
// estimates c_q that the next block subtracts from the microphones.
struct FcArgs {
  DevTier T;                 // its single tier (uniform partitions, P = B)
  const Item* items;         // its multiply-accumulate items (terms p >= 2)
  const Group* groups;       // its output groups (partial-slot layout)
  const void* H01;           // [Lf][Qf][2][P] its partitions 0 and 1
  float* hist;               // [Qf][hist_len] synthesis output history
  float* c;                  // [Lf][B] estimate c_{n-1}, written by its heads
  unsigned int* done;        // its heads done so far (monotonic, system scope)
  int64_t hist_mask;
  int32_t n_items;           // its items per launch
  int32_t tail0;             // tail index of its first item in the launch
  int32_t n_heads, head_slots;  // one head per feedback output; part of the grid
  int32_t Qf, Lf;            // its inputs (= synthesis outputs), outputs
  int32_t wait_polls;        // bound of the synthesis heads' wait for c
  uint32_t wait_bias;        // added to the wait's target (nonzero only to
                             // test the give-up path: never reached)
};

struct KArgs {
  DevTier tier[kMaxTiers];
  const Item* items;         // [n_phase][max_items]
  const int32_t* phase_count;
  const Group* groups;
  float* hist;               // input history [Q][hist_len]
  const float* in;           // [Q][B]
  float* out;                // [L][B]
  int64_t hist_mask;         // hist_len - 1
  int64_t ring_mask;         // output ring length - 1
  int32_t B, Q, L, n_tiers;
  int32_t n_phase, max_items;
  int32_t head_nq;           // inputs transformed per pass by a head
  int32_t n_head;            // head workgroups (one per output)
  int32_t head_slots;        // head part of the grid (n_head rounded up to 8)
  int32_t tails_wait;        // rta_process: multiply-accumulate workgroups
                             // start once this launch's heads are done
  int64_t n;                 // index of the block of this launch
  const Item* tier_items;    // later tiers' transform passes [n_phase][max_tier_items]
  const int32_t* tier_count; // transform items per phase
  const int32_t* tier_slot0; // [tier][group] first partial slot of later tiers
  const int32_t* tier_nslot; // [tier][group] partial slots of later tiers
  int32_t max_tier_items;
  int32_t n_groups_total;
  int32_t tier_slots;        // transform part of this launch's grid (a multiple of 8)
  int32_t pad4;
  unsigned int* heads_done;  // heads finished so far (monotonic, agent scope)
  const void* H01;           // [L][Q][2][P] spectra of partitions 0 and 1
  unsigned int* head_count;  // heads finished in this launch (zero between)
  int64_t* done_flag;        // host-visible: n + 1 once the output is written
  const float* sub;          // feedback estimate [Q][B] subtracted from `in`
  float* out2;               // second copy of the output block (feedback input)
  const int32_t* live;       // [Q] serving: 0 = the slot's input reads as zero
                             // (null: every input is live)
  int32_t fc_on;             // the feedback convolution runs in this launch
  int32_t nf3;               // n_f = 3 n_x: the heads hand their output spectra
                             // to the feedback convolution (no transform of y)
  int32_t* status;           // host-visible error word: a wait that gave up
                             // stores 1 (system scope); checked by the host
  const int64_t* n_base;     // graph replay: the block index is *n_base + n
                             // (null: n itself)
  FcArgs fc;
};

// ---------------------------------------------------------------------------
// Filter-spectrum element loads: C = 2 consecutive complex bins per lane and
// row, one non-temporal load (16 bytes of FP32 spectra, 8 bytes of 16-bit
// spectra).  Every type thus has the same lane -> bin mapping; the 16-bit
// types keep twice as many rows in flight for the same bytes.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

struct f16c_t { uint32_t bits; };   // packed (re, im) FP16 pair
struct bf16c_t { uint32_t bits; };  // packed (re, im) BF16 pair

template <typename HT> struct HVec;

template <> struct HVec<float2> {
  static constexpr int C = 2;
  static constexpr int U = kUnroll;
  typedef f32x4 raw_t;
  template <bool NT>
  static __device__ __forceinline__ raw_t load_raw(const float2* p) {
    if (NT) return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return *reinterpret_cast<const f32x4*>(p);
  }
  static __device__ __forceinline__ void unpack(const raw_t& v, float2 (&h)[C]) {
    h[0] = make_float2(v.x, v.y);
    h[1] = make_float2(v.z, v.w);
  }
  static __device__ __forceinline__ float2 load1(const float2* p) { return *p; }
  // one element as loaded, converted where it is used (held across other
  // work, a converted load would make the wave wait for it at once)
  typedef float2 one_t;
  static __device__ __forceinline__ one_t load1_raw(const float2* p) { return *p; }
  static __device__ __forceinline__ float2 cvt1(one_t v) { return v; }
};

__device__ __forceinline__ float2 f16pair(uint32_t w) {
  // the halves are taken apart as scalars: a vector bit_cast of a loaded
  // word here once made the compiler shrink the load and drop words
  const _Float16 re = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
  const _Float16 im = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  return make_float2((float)re, (float)im);
}

__device__ __forceinline__ float2 bf16pair(uint32_t w) {
  return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

template <> struct HVec<f16c_t> {
  static constexpr int C = 2;
  static constexpr int U = kUnroll16;
  typedef u32x2 raw_t;
  template <bool NT>
  static __device__ __forceinline__ raw_t load_raw(const f16c_t* p) {
    if (NT) return __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    return *reinterpret_cast<const u32x2*>(p);
  }
  static __device__ __forceinline__ void unpack(const raw_t& v, float2 (&h)[C]) {
    h[0] = f16pair(v.x);
    h[1] = f16pair(v.y);
  }
  static __device__ __forceinline__ float2 load1(const f16c_t* p) { return f16pair(p->bits); }
  typedef uint32_t one_t;
  static __device__ __forceinline__ one_t load1_raw(const f16c_t* p) { return p->bits; }
  static __device__ __forceinline__ float2 cvt1(one_t v) { return f16pair(v); }
};

template <> struct HVec<bf16c_t> {
  static constexpr int C = 2;
  static constexpr int U = kUnroll16;
  typedef u32x2 raw_t;
  template <bool NT>
  static __device__ __forceinline__ raw_t load_raw(const bf16c_t* p) {
    if (NT) return __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    return *reinterpret_cast<const u32x2*>(p);
  }
  static __device__ __forceinline__ void unpack(const raw_t& v, float2 (&h)[C]) {
    h[0] = bf16pair(v.x);
    h[1] = bf16pair(v.y);
  }
  static __device__ __forceinline__ float2 load1(const bf16c_t* p) { return bf16pair(p->bits); }
  typedef uint32_t one_t;
  static __device__ __forceinline__ one_t load1_raw(const bf16c_t* p) { return p->bits; }
  static __device__ __forceinline__ float2 cvt1(one_t v) { return bf16pair(v); }
};

// Prefetched values are pinned where they are used: the empty asm takes the
// register as it is, so the compiler cannot move arithmetic on the value up
// to its load (where the wave would then wait for the load to return).
__device__ __forceinline__ float pin(float v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ uint32_t pin(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ int pin(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ float2 pin(float2 v) { return make_float2(pin(v.x), pin(v.y)); }

__device__ __forceinline__ int wrap_slot(int64_t v, int K) {
  int s = (int)(v % K);
  return s < 0 ? s + K : s;
}

// ---------------------------------------------------------------------------
// Multiply-accumulate of one item's partitions into its partial-sum slot.
// `frame` is the frame whose delay-line head is slot frame mod K (partition
// p pairs with slot (frame - p) mod K).
// ---------------------------------------------------------------------------
template <typename HT, int G, bool NT>
__device__ __forceinline__ void mac_item(const DevTier& T, const Item& it, int64_t frame, float2* red) {
  constexpr int C = HVec<HT>::C;
  const int P = T.P;
  const int W = it.w;                                  // bins per item slice
  const int LR = W / C;                                // lanes per row
  const int RP = kThreads / LR;                        // rows per pass
  const int tid = threadIdx.x;
  const int r = tid % LR, s = tid / LR;
  const int kb = it.k0 + r * C;
  const int q = it.q;
  const HT* Hbase = reinterpret_cast<const HT*>(T.H);

  const HT* hb[G];
  int pend[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const bool on = g < it.nl;
    pend[g] = on ? it.pend[g] : 0;
    hb[g] = Hbase + (on ? it.row[g] : 0) * (int64_t)P + kb;
  }

  float acc[G][C][4];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < C; ++j) acc[g][j][0] = acc[g][j][1] = acc[g][j][2] = acc[g][j][3] = 0.f;

  const int K = T.K;
  const float2* Xq = T.X + (int64_t)q * K * P + kb;
  const int step = RP % K;
  int p = it.p0 + s;
  int slot = wrap_slot(frame - p, K);
  // U rows in flight per lane: every load of a pass is issued before any
  // is used (raw registers), then the pass is accumulated
  constexpr int U = HVec<HT>::U;
  typedef typename HVec<HT>::raw_t raw_t;
  for (; p < it.p1; p += RP * U) {
    f32x4 xr[U];
    raw_t hr[U][G];
    int sl = slot;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int pu = p + u * RP;
      xr[u] = pu < it.p1 ? *reinterpret_cast<const f32x4*>(Xq + (int64_t)sl * P) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int g = 0; g < G; ++g)
        hr[u][g] = pu < pend[g] ? HVec<HT>::template load_raw<NT>(hb[g] + (int64_t)pu * P) : raw_t{};
      sl -= step;
      if (sl < 0) sl += K;
    }
    slot = sl;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float2 xv[C] = {make_float2(xr[u].x, xr[u].y), make_float2(xr[u].z, xr[u].w)};
#pragma unroll
      for (int g = 0; g < G; ++g) {
        float2 hv[C];
        HVec<HT>::unpack(hr[u][g], hv);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          acc[g][j][0] += hv[j].x * xv[j].x;   // Re H Re X
          acc[g][j][1] += hv[j].y * xv[j].y;   // Im H Im X
          acc[g][j][2] += hv[j].x * xv[j].y;   // Re H Im X
          acc[g][j][3] += hv[j].y * xv[j].x;   // Im H Re X
        }
      }
    }
  }

  // combine the four real sums; packed bin 0 holds two real products
  float2 res[G][C];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < C; ++j) {
      if (kb + j == 0)
        res[g][j] = make_float2(acc[g][j][0], acc[g][j][1]);
      else
        res[g][j] = make_float2(acc[g][j][0] - acc[g][j][1], acc[g][j][2] + acc[g][j][3]);
    }

  // later tiers: chunks of one (group, input) accumulated in earlier blocks
  // of the frame share the slot; the first stored it
  float2* part = T.partial + (int64_t)it.slot * G * P;
  if (RP == 1) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < C; ++j) {
        float2* d = part + (int64_t)g * P + kb + j;
        *d = it.acc ? cadd(*d, res[g][j]) : res[g][j];
      }
    return;
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < C; ++j) red[(s * G + g) * W + r * C + j] = res[g][j];
  __syncthreads();
  for (int e = tid; e < G * W; e += kThreads) {
    const int g = e / W, b = e - g * W;
    float2 sum = red[g * W + b];
    for (int s2 = 1; s2 < RP; ++s2) sum = cadd(sum, red[(s2 * G + g) * W + b]);
    float2* d = part + (int64_t)g * P + it.k0 + b;
    *d = it.acc ? cadd(*d, sum) : sum;
  }
}

// Thread split of a reduction over E elements per input (bins, or bins of
// several outputs): the 256 threads form kThreads / span groups, span the
// largest power of two dividing E (at most 256), and each thread covers the
// E / span elements tid mod span + i span (3 of them for the 3 * 2^m bins
// of n_f = 3B, none idle); LDS scratch of 256 * E / span float2 combines the
// groups in group order (reproducible).
__host__ __device__ constexpr int red_span(int E) { return (E & -E) < kThreads ? (E & -E) : kThreads; }
__host__ __device__ constexpr int red_scratch(int E) { return red_span(E) == kThreads ? kThreads : kThreads * (E / red_span(E)); }

// Twiddle tables of tiers up to this size are staged in LDS before an FFT;
// larger ones are read from global memory (they stay hot in L1/L2).
constexpr int kTwLdsMaxP = 1024;
__host__ __device__ constexpr int tw_lds_len(int P) { return P <= kTwLdsMaxP ? 2 * P : 0; }

// Twiddles of tables up to kThreads * kTwRegs entries are loaded into
// registers first and written to LDS later (stage_twiddles_regs /
// store_twiddles_regs), so their global round trip overlaps the head's other
// loads instead of preceding them.
constexpr int kTwRegs = 2;
struct TwRegs { float2 v[kTwRegs]; int n; };
__device__ __forceinline__ TwRegs load_twiddles_regs(const DevTier& T) {
  TwRegs r;
  r.n = tw_lds_len(T.P);
  if (r.n > kTwRegs * kThreads) r.n = 0;  // too long: stage_twiddles instead
  // unconditional loads at clamped indices (a load under a lane-divergent
  // guard makes the wave wait for every load in flight)
#pragma unroll
  for (int i = 0; i < kTwRegs; ++i)
    if (i * kThreads < r.n) r.v[i] = T.tw[min((int)threadIdx.x + i * kThreads, r.n - 1)];
  return r;
}
__device__ __forceinline__ void store_twiddles_regs(const TwRegs& r, float2* dst) {
#pragma unroll
  for (int i = 0; i < kTwRegs; ++i) {
    const int j = threadIdx.x + i * kThreads;
    if (j < r.n) dst[j] = pin(r.v[i]);
  }
}

// Returns the twiddle table to use: a copy in LDS at `dst` when it fits,
// otherwise the global table.  No barrier: the caller's next barrier
// publishes the copy.
__device__ __forceinline__ const float2* stage_twiddles(const DevTier& T, float2* dst) {
  const int n = tw_lds_len(T.P);
  if (n == 0) return T.tw;
  for (int i = threadIdx.x; i < n; i += kThreads) dst[i] = T.tw[i];
  return dst;
}

// Sum the first tier's partial slots of a whole output group, all its
// outputs at once (elements e = g P + k are contiguous within a slot), and
// add the p = 1 term sum_q H_{l,q,1} X_q(n-1), which needs no new spectrum.
// When 256 does not divide into whole passes over the E elements (E < 256,
// or E = 3 * 2^m), the threads form groups (red_span) that each add a
// contiguous run of slots, combined in group order (fixed for given E and
// nslot, so results are reproducible).  Y: [G][P] in LDS; scratch:
// red_scratch(E) float2.  Ends with a barrier.
template <typename HT, int G>
__device__ __forceinline__ void head_reduce(const KArgs& A, const DevTier& T, const Group& grp, int64_t n,
                            float2* Y, float2* scratch) {
  const int P = T.P;
  const int E = grp.nl * P;
  const int64_t stride = (int64_t)G * P;
  const float2* base = T.partial + (int64_t)grp.slot0 * stride;
  const int tid = threadIdx.x;
  const bool has_p1 = T.K >= 2;
  const int slot1 = wrap_slot(n - 1, T.K);
  const HT* H01 = reinterpret_cast<const HT*>(A.H01);
  // inputs q0, q0 + dq, ... of the p = 1 term of element e
  auto p1_term = [&](int e, int q0, int dq) {
    float2 t = make_float2(0.f, 0.f);
    if (!has_p1) return t;
    const int g = e / P, k = e - g * P;
    const int l = grp.l0 + g;
#pragma unroll 4
    for (int q = q0; q < A.Q; q += dq) {
      const float2 h1 = HVec<HT>::load1(H01 + ((int64_t)(l * A.Q + q) * 2 + 1) * P + k);
      const float2 x1 = T.X[((int64_t)q * T.K + slot1) * P + k];
      t = cadd(t, (k == 0) ? make_float2(h1.x * x1.x, h1.y * x1.y) : cmul(h1, x1));
    }
    return t;
  };
  const int span = red_span(E);
  if (span == kThreads) {
    for (int e = tid; e < E; e += kThreads) {
      float2 acc = p1_term(e, 0, 1);
#pragma unroll 16
      for (int sl = 0; sl < grp.nslot; ++sl) acc = cadd(acc, base[sl * stride + e]);
      Y[e] = acc;
    }
    __syncthreads();
    return;
  }
  const int ng = kThreads / span, tg = tid / span;
  const int per = (grp.nslot + ng - 1) / ng;
  const int s0 = min(grp.nslot, tg * per), s1 = min(grp.nslot, s0 + per);
  for (int e = tid % span; e < E; e += span) {
    float2 acc = p1_term(e, tg, ng);  // the thread groups split the inputs
#pragma unroll 16
    for (int sl = s0; sl < s1; ++sl) acc = cadd(acc, base[sl * stride + e]);
    scratch[tg * E + e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < E; e += kThreads) {
    float2 t = scratch[e];
    for (int g2 = 1; g2 < ng; ++g2) t = cadd(t, scratch[g2 * E + e]);
    Y[e] = t;
  }
  __syncthreads();
}

// The same reduction split in two, so that its global round trip overlaps
// the head's transform of the block's window (which does not depend on it):
// red_issue() requests every value one thread adds -- its run of partial
// slots of its one element and the operands of its share of the p = 1 term
// -- into registers, red_finish() adds them into Y after the transform.
// Only for element counts E that are powers of two up to 256 (one element
// per thread, red_span(E) = E) and per-thread shares within the register
// budget (red_fits); other shapes take head_reduce().
template <typename HT>
struct HeadRed {
  static constexpr int kSlots = 16, kInputs = 4;
  float2 s[kSlots];
  typename HVec<HT>::one_t h1[kInputs];
  float2 x1[kInputs];
};
__device__ __forceinline__ bool red_fits(int E, int nslot, int Q, int HRslots, int HRinputs) {
  if (E > kThreads || (E & (E - 1)) != 0) return false;
  const int ng = kThreads / E;
  return (nslot + ng - 1) / ng <= HRslots && (Q + ng - 1) / ng <= HRinputs;
}
template <typename HT, int G>
__device__ __forceinline__ void red_issue(const KArgs& A, const DevTier& T, const Group& grp,
                                          int64_t n, HeadRed<HT>& r, bool on) {
  const int P = T.P;
  const int E = grp.nl * P;
  const int64_t stride = (int64_t)G * P;
  const float2* base = T.partial + (int64_t)grp.slot0 * stride;
  const int tid = threadIdx.x;
  // (off the split path E may exceed kThreads; the loads then all read the
  // dummy address and these only have to be defined)
  const int ng = max(1, kThreads / E), tg = tid / E, e = tid % E;
  const int per = (grp.nslot + ng - 1) / ng;
  const int s0 = min(grp.nslot, tg * per);
  // Always kSlots loads, at clamped indices (a valid dummy address when the
  // group has no slots, or when the reduction is not split: on = false),
  // with no guard: the compiler then knows that at least kSlots loads follow
  // the window's and waits for the window alone (with a guarded or variable
  // count it waits for every load in flight).  red_finish adds only the
  // thread's own slots.
  const bool any = on && grp.nslot > 0;
  const float2* src = any ? base + e : T.tw;
  const int64_t step = any ? stride : 0;
  const int last = max(grp.nslot - 1, 0);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < HeadRed<HT>::kSlots; ++i) r.s[i] = src[min(s0 + i, last) * step];
  if (!on || T.K < 2) return;
  const int slot1 = wrap_slot(n - 1, T.K);
  const HT* H01 = reinterpret_cast<const HT*>(A.H01);
  const int g = e / P, k = e - g * P;
  const int l = grp.l0 + g;
  const int nq = (A.Q + ng - 1) / ng;
#pragma unroll
  for (int j = 0; j < HeadRed<HT>::kInputs; ++j) {
    if (j < nq) {
      const int q = min(tg + j * ng, A.Q - 1);
      r.h1[j] = HVec<HT>::load1_raw(H01 + ((int64_t)(l * A.Q + q) * 2 + 1) * P + k);
      r.x1[j] = T.X[((int64_t)q * T.K + slot1) * P + k];
    }
  }
}
// Y [E] in LDS; scratch: kThreads float2.  Every thread's element is its own
// (e = tid for tid < E) when this returns; no barrier after the last write.
template <typename HT, int G>
__device__ __forceinline__ void red_finish(const KArgs& A, const DevTier& T, const Group& grp,
                                           const HeadRed<HT>& r, float2* Y, float2* scratch) {
  const int P = T.P;
  const int E = grp.nl * P;
  const int tid = threadIdx.x;
  const int ng = kThreads / E, tg = tid / E, e = tid % E;
  const int per = (grp.nslot + ng - 1) / ng;
  const int s0 = min(grp.nslot, tg * per), s1 = min(grp.nslot, s0 + per);
  const int k = e % P;
  float2 acc = make_float2(0.f, 0.f);
  if (T.K >= 2) {
    const int nq = (A.Q + ng - 1) / ng;
#pragma unroll
    for (int j = 0; j < HeadRed<HT>::kInputs; ++j) {
      if (j < nq && tg + j * ng < A.Q) {
        const float2 h1 = HVec<HT>::cvt1(pin(r.h1[j]));
        const float2 x1 = pin(r.x1[j]);
        acc = cadd(acc, (k == 0) ? make_float2(h1.x * x1.x, h1.y * x1.y) : cmul(h1, x1));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < HeadRed<HT>::kSlots; ++i)
    if (i < per && s0 + i < s1) acc = cadd(acc, pin(r.s[i]));
  if (ng == 1) {
    Y[e] = acc;
    return;
  }
  scratch[tg * E + e] = acc;
  __syncthreads();
  if (tid < E) {
    float2 t = scratch[tid];
    for (int g2 = 1; g2 < ng; ++g2) t = cadd(t, scratch[g2 * E + tid]);
    Y[tid] = t;
  }
}

// Fused feedback: thread 0 waits until every feedback head of this launch
// has published c_{n-1} (they are dispatched first and wait for nothing),
// then the workgroup proceeds.  The spin is bounded all the same; a wait that
// gives up stores 1 in the host-visible error word, which fails the block on
// the host.
__device__ void fc_wait(const KArgs& A, int64_t n) {
  if (threadIdx.x == 0) {
    const unsigned int target = (unsigned int)((n + 1) * A.fc.n_heads) + A.fc.wait_bias;
    bool ready = false;
    for (int it = 0; it < A.fc.wait_polls; ++it) {
      if ((int)(__hip_atomic_load(A.fc.done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) - target) >= 0) {
        ready = true;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ready) __hip_atomic_store(A.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __syncthreads();
}

// LDS layout of a head workgroup, in float2 units (the host sizes the launch with the
// same function): Y [G][P] | Xa [nbuf][P] | Xb [nbuf][P] | twiddles | 256.
struct HeadLds {
  int y, xa, xb, tw, scratch, total;
};
__host__ __device__ inline HeadLds head_lds(int P, int G, int nq) {
  const int nbuf = nq > G ? nq : G;
  HeadLds h;
  h.y = 0;
  h.xa = G * P;
  h.xb = h.xa + nbuf * P;
  h.tw = h.xb + nbuf * P;
  h.scratch = h.tw + tw_lds_len(P);
  h.total = h.scratch + red_scratch(P);
  return h;
}

// Head workgroup of block n for one output: `grp` is the single-output group
// {l, 1} and gsel the output's index within its tail group of G outputs (its
// row in every partial slot).  One head per output keeps each head's share
// of the partial-sum reduction, the critical path under the tails' streaming,
// independent of G.
template <typename HT, int G>
__device__ __forceinline__ void head_work(const KArgs& A, int64_t n, const Group& grp, int gsel, float2* lds) {
  const int tid = threadIdx.x;
  const DevTier& T = A.tier[0];
  // P bins per row, half the window of 2P samples: P = B (n_f = 2B), or
  // P = 3B/2 (n_f = 3B, T.r3)
  const int P = T.P, logP = T.logP;
  const HeadLds L = head_lds(P, 1, A.head_nq);
  float2* Y = lds + L.y;
  float2* Xa = lds + L.xa;
  float2* Xb = lds + L.xb;
  float2* scratch = lds + L.scratch;
  // twiddles for the FFTs: requested now, written to LDS after the partial-sum
  // reduction (its loads then share the round trip); published by the
  // barrier before the first FFT
  {
    // the prologue's kernel-argument fields in one batch (as in k_block)
    const void* p0 = A.hist;
    const void* p1 = A.in;
    const void* p2 = A.sub;
    const void* p3 = A.live;
    const void* p4 = A.H01;
    const void* p5 = A.tier[1].oring;
    const void* p6 = A.tier[2].oring;
    const int64_t m0 = A.hist_mask, m1 = A.ring_mask;
    const int i0 = A.head_nq, i1 = A.Q, i2 = A.B, i3 = A.fc_on, i4 = A.n_tiers;
    asm volatile("" ::"s"(T.tw), "s"(T.X), "s"(T.partial), "s"(T.K), "s"(T.P), "s"(T.logP), "s"(T.r3),
                 "s"(T.nslots), "s"(p0), "s"(p1), "s"(p2), "s"(p3), "s"(p4), "s"(p5), "s"(p6), "s"(m0), "s"(m1),
                 "s"(i0), "s"(i1), "s"(i2), "s"(i3), "s"(i4));
  }
  const TwRegs twr = load_twiddles_regs(T);
  const float2* tw = twr.n > 0 ? lds + L.tw : stage_twiddles(T, lds + L.tw);
  const HT* H01 = reinterpret_cast<const HT*>(A.H01);

  // 0. Prefetch.  The heads run beside the bandwidth-bound tails, so every
  //    global round trip is slow; everything that does not depend on this
  //    block's FFT is requested up front into registers -- the first input
  //    chunk's window samples and H_{l,q,0} coefficients, and the later
  //    tiers' ring samples of this block -- so that its latency overlaps the
  //    partial-sum loads of step 1.  (Sizes beyond the register budget fall
  //    back to loading in place.)
  constexpr int WMAX = 2, HMAX = 4, RMAX = 1, TMAX = 2;
  const int E = grp.nl * P;
  const int nb0 = min(A.head_nq, A.Q);
  const int ept = (E + kThreads - 1) / kThreads;       // output elements per thread
  const int hb = A.B >> 1;                              // sample pairs per output block
  const int m0 = P - hb;                                // its first complex sample
  const int eo = grp.nl * hb;                           // output sample pairs
  const int cur = 2 * P - A.B;                          // window samples from the history
  const int64_t wh0 = (n + 1) * A.B - 2 * (int64_t)P;   // stream index of window sample 0
  // (fused feedback: the window needs c_{n-1}, which this launch's feedback
  // heads are still computing, so it is not prefetched)
  const bool pre_w = nb0 * P <= WMAX * kThreads && !A.fc_on;
  const bool pre_h = ept * nb0 <= HMAX;
  const bool pre_r = A.n_tiers - 1 <= TMAX && eo <= RMAX * kThreads;
  // Window sample pair m of input q, [w_2m, w_2m+1]: both from the history
  // (2m < cur) or both from this block's input (cur is even).  The source is
  // selected per lane and read with unconditional loads (clamped indices,
  // guards applied where the values are used): a load under a lane-divergent
  // branch makes the wave wait for every load in flight, which would undo
  // the prefetch.
  struct WinRaw {
    float2 w, s;  // samples; the feedback estimate of input samples
    int live;
  };
  auto win_load = [&](int e, int q0) {
    const int b = e / P, m = e - b * P;
    const int q = q0 + b;
    const int i0 = 2 * m;
    const float* p = i0 < cur ? A.hist + (int64_t)q * (A.hist_mask + 1) + ((wh0 + i0) & A.hist_mask)
                              : A.in + (int64_t)q * A.B + (i0 - cur);
    WinRaw r;
    r.w = make_float2(p[0], p[1]);
    r.s = make_float2(0.f, 0.f);
    if (A.sub != nullptr) {  // microphone minus the previous block's feedback estimate
      const float* ps = A.sub + (int64_t)q * A.B + max(i0 - cur, 0);
      // (fused: written in this launch by another workgroup, so read where
      // every XCD sees it)
      r.s = A.fc_on ? make_float2(__hip_atomic_load(ps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM),
                                  __hip_atomic_load(ps + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
                    : make_float2(ps[0], ps[1]);
    }
    r.live = A.live != nullptr ? A.live[q] : 1;
    return r;
  };
  auto win_value = [&](int e, const WinRaw& r) {
    if (2 * (e % P) < cur) return r.w;
    const float2 v = make_float2(r.w.x - r.s.x, r.w.y - r.s.y);
    return r.live == 0 ? make_float2(0.f, 0.f) : v;  // a select: NaN input stays out
  };
  auto h0_at = [&](int e, int q) {
    const int g = e / P, k = e - g * P;
    return HVec<HT>::load1(H01 + ((int64_t)((grp.l0 + g) * A.Q + q) * 2) * P + k);
  };
  WinRaw wv[WMAX];
  typename HVec<HT>::one_t hv[HMAX];
  float rv[RMAX][TMAX][2];
  if (pre_w) {
#pragma unroll
    for (int i = 0; i < WMAX; ++i)
      if (i * kThreads < nb0 * P) wv[i] = win_load(min(tid + i * kThreads, nb0 * P - 1), 0);
  }
  __builtin_amdgcn_sched_barrier(0);  // the window's loads go out first
  if (pre_h) {
#pragma unroll
    for (int i = 0; i < HMAX; ++i) {
      const int ie = i / nb0, b = i - ie * nb0;
      if (ie < ept) {
        const int e = min(tid + ie * kThreads, E - 1);
        const int g = e / P, k = e - g * P;
        hv[i] = HVec<HT>::load1_raw(H01 + ((int64_t)((grp.l0 + g) * A.Q + b) * 2) * P + k);
      }
    }
  }
  if (pre_r) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      const int e = min(tid + i * kThreads, eo - 1);
#pragma unroll
      for (int t = 0; t < TMAX; ++t) {
        if (i * kThreads < eo && t + 1 < A.n_tiers) {
          const int g = e / hb, j = 2 * (e - g * hb);
          const float* ring = A.tier[t + 1].oring + (int64_t)(grp.l0 + g) * (A.ring_mask + 1);
          rv[i][t][0] = ring[(n * A.B + j) & A.ring_mask];
          rv[i][t][1] = ring[(n * A.B + j + 1) & A.ring_mask];
        }
      }
    }
  }

  // 1. the terms p >= 2, summed by the previous launch's tail items, and the
  //    term p = 1 (ring slot n-1): requested now and added up after the
  //    window's transform (step 2) where the shape allows, else done here
  const DevTier Tcur = [&] {
    DevTier t = T;
    t.partial = T.partial + (n & 1) * (int64_t)T.nslots * G * P + (int64_t)gsel * P;
    return t;
  }();
  HeadRed<HT> red;
  const bool split = red_fits(E, grp.nslot, A.Q, HeadRed<HT>::kSlots, HeadRed<HT>::kInputs);
  // (issued on both paths: one straight-line sequence of loads after the
  // window's, whatever the shape)
  red_issue<HT, G>(A, Tcur, grp, n, red, split);
  if (!split) {
    head_reduce<HT, G>(A, Tcur, grp, n, Y, scratch);
    // nothing left in flight on this path, so that the compiler's count of
    // loads still outstanding where the paths meet is the split path's
    __builtin_amdgcn_s_waitcnt(0);
  }
  store_twiddles_regs(twr, lds + L.tw);

  // fused feedback: wait until every feedback head of this launch has
  // published c_{n-1}
  if (A.fc_on) fc_wait(A, n);

  // 2. the term p = 0: window -> real FFT -> ring slot n mod K, times H_{l,q,0}
  const int slot0 = wrap_slot(n, T.K);
  // window sample pair e of inputs q0, q0 + 1, ... into LDS; the first group
  // also stores the block's input samples (as windowed: feedback estimate
  // subtracted, silent inputs zero) into the history for later launches
  auto put = [&](int q0, int e, float2 v) {
    Xa[e] = v;
    const int bq = e / P, i = 2 * (e - bq * P) - cur;
    if (grp.l0 == 0 && i >= 0) {
      float* h = A.hist + (int64_t)(q0 + bq) * (A.hist_mask + 1);
      h[(n * A.B + i) & A.hist_mask] = v.x;
      h[(n * A.B + i + 1) & A.hist_mask] = v.y;
    }
  };
  // the windows of nb inputs from q0 in LDS -> real FFT -> ring slot n mod
  // K; the term p = 0 added into Y (first: the chunk the prefetch covered,
  // which also adds up the split reduction first)
  auto chunk = [&](int q0, int nb, bool first) {
    __syncthreads();
    float2* z = fft_any<false>(Xa, Xb, P, logP, T.r3, tw, nb);
    float2* x = (z == Xa) ? Xb : Xa;
    rfft_post(z, x, P, tw + P, nb);
    if (grp.l0 == 0) {  // the first group stores the block's spectrum for later launches
      for (int e = tid; e < nb * P; e += kThreads) {
        const int b = e / P, k = e - b * P;
        T.X[((int64_t)(q0 + b) * T.K + slot0) * P + k] = x[e];
      }
    }
    // the reduction's registers into Y (element e = tid, as below)
    if (first && split) red_finish<HT, G>(A, Tcur, grp, red, Y, scratch);
    if (first && pre_h) {
      // register slot i holds element ie = i / nb, input b = i % nb (the
      // same mapping as the prefetch); each element belongs to this thread
#pragma unroll
      for (int i = 0; i < HMAX; ++i) {
        const int ie = i / nb, b = i - ie * nb;
        const int e = tid + ie * kThreads;
        if (ie >= ept || e >= E) continue;
        const int k = e % P;
        const float2 h0 = HVec<HT>::cvt1(pin(hv[i]));
        const float2 x0 = x[b * P + k];
        Y[e] = cadd(Y[e], (k == 0) ? make_float2(h0.x * x0.x, h0.y * x0.y) : cmul(h0, x0));
      }
    } else {
      for (int e = tid; e < E; e += kThreads) {
        const int k = e % P;
        float2 acc = Y[e];
#pragma unroll 4
        for (int b = 0; b < nb; ++b) {
          const float2 h0 = h0_at(e, q0 + b);
          const float2 x0 = x[b * P + k];
          acc = cadd(acc, (k == 0) ? make_float2(h0.x * x0.x, h0.y * x0.y) : cmul(h0, x0));
        }
        Y[e] = acc;
      }
    }
    __syncthreads();
  };
  // first chunk, from the prefetched registers where it was prefetched (kept
  // out of the loop below: the compiler then waits for these loads alone)
  if (pre_w) {
#pragma unroll
    for (int i = 0; i < WMAX; ++i) {
      const int e = tid + i * kThreads;
      if (e < nb0 * P) {
        WinRaw r = wv[i];
        r.w = pin(r.w);
        r.s = pin(r.s);
        r.live = pin(r.live);
        put(0, e, win_value(e, r));
      }
    }
  } else {
    for (int e = tid; e < nb0 * P; e += kThreads) put(0, e, win_value(e, win_load(e, 0)));
  }
  chunk(0, nb0, true);
  for (int q0 = A.head_nq; q0 < A.Q; q0 += A.head_nq) {
    const int nb = min(A.head_nq, A.Q - q0);
    for (int e = tid; e < nb * P; e += kThreads) put(q0, e, win_value(e, win_load(e, q0)));
    chunk(q0, nb, false);
  }

  // n_f = 3B (Sec. V): this output's accumulated spectrum is the spectrum
  // of a 3B-sample frame whose last 2B samples are [y_l(n-1), y_l(n)], all
  // the feedback filters' B-tap partitions need, so it goes into slot n of
  // the feedback delay line as it is -- no inverse-then-forward transform
  if (A.fc_on && A.nf3) {
    const FcArgs& F = A.fc;
    float2* dst = F.T.X + ((int64_t)grp.l0 * F.T.K + wrap_slot(n, F.T.K)) * P;
    for (int k = tid; k < P; k += kThreads) dst[k] = Y[k];
  }

  // 3. inverse real FFT of the group's outputs, keep the last B samples, add
  //    the later tiers' contributions from their output rings (and clear
  //    them), emit
  irfft_pre(Y, Xa, P, tw + P, grp.nl);
  float2* z = fft_any<true>(Xa, Xb, P, logP, T.r3, tw, grp.nl);
  const float scale = 1.0f / (float)(2 * P);
  auto emit = [&](int e, float y0, float y1) {
    const int g = e / hb, m = m0 + (e - g * hb);
    const int l = grp.l0 + g;
    const int i = 2 * (m - m0);
    const float2 v = z[g * P + m];
    const float o0 = y0 + v.x * scale, o1 = y1 + v.y * scale;
    A.out[(int64_t)l * A.B + i] = o0;
    A.out[(int64_t)l * A.B + i + 1] = o1;
    if (A.out2 != nullptr) {
      A.out2[(int64_t)l * A.B + i] = o0;
      A.out2[(int64_t)l * A.B + i + 1] = o1;
    }
    if (A.fc_on) {  // kept for the feedback hand-off (one output per head)
      reinterpret_cast<float*>(Y)[i] = o0;
      reinterpret_cast<float*>(Y)[i + 1] = o1;
    }
  };
  auto clear_rings = [&](int e) {
    const int g = e / hb, j = 2 * (e - g * hb);
    for (int t = 1; t < A.n_tiers; ++t) {
      float* ring = A.tier[t].oring + (int64_t)(grp.l0 + g) * (A.ring_mask + 1);
      ring[(n * A.B + j) & A.ring_mask] = 0.f;
      ring[(n * A.B + j + 1) & A.ring_mask] = 0.f;
    }
  };
  if (pre_r) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      const int e = tid + i * kThreads;
      if (e >= eo) continue;
      float y0 = 0.f, y1 = 0.f;
#pragma unroll
      for (int t = 0; t < TMAX; ++t) {
        if (t + 1 < A.n_tiers) {
          y0 += pin(rv[i][t][0]);
          y1 += pin(rv[i][t][1]);
        }
      }
      emit(e, y0, y1);
      clear_rings(e);
    }
  } else {
    for (int e = tid; e < eo; e += kThreads) {
      const int g = e / hb, j = 2 * (e - g * hb);
      float y0 = 0.f, y1 = 0.f;
      for (int t = 1; t < A.n_tiers; ++t) {
        const float* ring = A.tier[t].oring + (int64_t)(grp.l0 + g) * (A.ring_mask + 1);
        y0 += ring[(n * A.B + j) & A.ring_mask];
        y1 += ring[(n * A.B + j + 1) & A.ring_mask];
      }
      emit(e, y0, y1);
      clear_rings(e);
    }
  }

  // this head's output is out: the tail workgroups of a waiting launch may
  // start streaming (relaxed: they read nothing the heads wrote)
  if (tid == 0) __hip_atomic_fetch_add(A.heads_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  // 4. completion (rta_process only): every head makes its output visible
  //    system-wide, the last one raises the flag (only the heads count, so
  //    the host does not wait for the tail workgroups of this launch)
  if (A.done_flag != nullptr) {
    __threadfence_system();
    __syncthreads();
    if (tid == 0) {
      const unsigned int old = __hip_atomic_fetch_add(A.head_count, 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_SYSTEM);
      if (old == (unsigned int)A.n_head - 1u) {
        __hip_atomic_store(A.head_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(A.done_flag, n + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }

  // 5. fused feedback: this output is input l of the feedback convolution;
  //    its window [y_l(n-1), y_l(n)] is transformed here, where y_l(n) already
  //    is, into the feedback delay line (slot n), and y_l(n) goes to its
  //    history -- the feedback launch needs no transform of its own
  if (!A.fc_on || A.nf3) return;
  __syncthreads();
  {
    const FcArgs& F = A.fc;
    const int l = grp.l0;
    const float* yn = reinterpret_cast<const float*>(Y);
    float* hl = F.hist + (int64_t)l * (F.hist_mask + 1);
    for (int m = tid; m < P; m += kThreads) {
      const int i0 = 2 * m, i1 = 2 * m + 1;
      const float w0 = i0 < P ? hl[((n - 1) * A.B + i0) & F.hist_mask] : yn[i0 - P];
      const float w1 = i1 < P ? hl[((n - 1) * A.B + i1) & F.hist_mask] : yn[i1 - P];
      Xa[m] = make_float2(w0, w1);
    }
    __syncthreads();
    for (int i = tid; i < A.B; i += kThreads) hl[(n * A.B + i) & F.hist_mask] = yn[i];
    float2* zf = fft_any<false>(Xa, Xb, P, logP, 0, tw);
    float2* xf = (zf == Xa) ? Xb : Xa;
    rfft_post(zf, xf, P, tw + P);
    float2* dst = F.T.X + ((int64_t)l * F.T.K + wrap_slot(n, F.T.K)) * P;
    for (int k = tid; k < P; k += kThreads) dst[k] = xf[k];
  }
}

// Feedback head of the fused launch n: output j of the feedback convolution
// for block n - 1, c_j = IFFT(sum of its partial slots (its items of launch
// n - 1) + sum_l F_{j,l,1} Y'_l(n-2) + F_{j,l,0} Y'_l(n-1)), the second half
// of the 2B samples; then it counts itself done (system scope, after making
// c visible).  Y' are the synthesis heads' transforms of their outputs.
template <typename HT, int G>
__device__ __forceinline__ void fc_head_work(const KArgs& A, int64_t n, int j, float2* lds) {
  const FcArgs& F = A.fc;
  const DevTier& T = F.T;
  const int P = T.P, logP = T.logP, tid = threadIdx.x;
  const Group g0 = F.groups[j / G];
  const int gsel = j - g0.l0;
  float2* Y = lds;
  float2* Xa = lds + P;
  float2* Xb = lds + 2 * P;
  float2* scratch = lds + 3 * P + tw_lds_len(P);  // red_scratch(P) float2
  // twiddles requested with the reduction's loads, written to LDS before its
  // closing barrier
  const TwRegs twr = load_twiddles_regs(T);
  const float2* tw = twr.n > 0 ? lds + 3 * P : stage_twiddles(T, lds + 3 * P);
  const HT* H01 = reinterpret_cast<const HT*>(F.H01);
  const int64_t stride = (int64_t)G * P;
  const float2* base = T.partial + ((n - 1) & 1) * (int64_t)T.nslots * G * P +
                       (int64_t)g0.slot0 * stride + (int64_t)gsel * P;
  const int s1 = wrap_slot(n - 1, T.K), s2 = wrap_slot(n - 2, T.K);
  auto term = [&](int k, int q0, int dq) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 4
    for (int q = q0; q < F.Qf; q += dq) {
      const HT* hr = H01 + ((int64_t)(j * F.Qf + q) * 2) * P + k;
      const float2 h0 = HVec<HT>::load1(hr), h1 = HVec<HT>::load1(hr + P);
      const float2 x0 = T.X[((int64_t)q * T.K + s1) * P + k];
      const float2 x1 = T.X[((int64_t)q * T.K + s2) * P + k];
      if (k == 0)
        acc = cadd(acc, make_float2(h0.x * x0.x + h1.x * x1.x, h0.y * x0.y + h1.y * x1.y));
      else
        acc = cadd(acc, cadd(cmul(h0, x0), cmul(h1, x1)));
    }
    return acc;
  };
  // threads split into groups over inputs and slots (red_span), each
  // covering P / span bins
  const int span = red_span(P);
  const int ng = kThreads / span, tg = tid / span;
  const int per = (g0.nslot + ng - 1) / ng;
  const int a0 = min(g0.nslot, tg * per), a1 = min(g0.nslot, a0 + per);
  for (int k = tid % span; k < P; k += span) {
    float2 acc = term(k, tg, ng);
#pragma unroll 8
    for (int sl = a0; sl < a1; ++sl) acc = cadd(acc, base[sl * stride + k]);
    if (ng == 1) Y[k] = acc; else scratch[tg * P + k] = acc;
  }
  store_twiddles_regs(twr, lds + 3 * P);
  __syncthreads();
  if (ng > 1) {
    for (int k = tid; k < P; k += kThreads) {
      float2 t = scratch[k];
      for (int g2 = 1; g2 < ng; ++g2) t = cadd(t, scratch[g2 * P + k]);
      Y[k] = t;
    }
    __syncthreads();
  }
  irfft_pre(Y, Xa, P, tw + P);
  float2* z = fft_any<true>(Xa, Xb, P, logP, T.r3, tw);
  const float scale = 1.0f / (float)(2 * P);
  const int m0 = P - (A.B >> 1);  // the last B of the 2P samples
  float* cj = F.c + (int64_t)j * A.B;
  for (int m = m0 + tid; m < P; m += kThreads) {
    const int i = 2 * (m - m0);
    __hip_atomic_store(cj + i, z[m].x * scale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(cj + i + 1, z[m].y * scale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __threadfence_system();
  __syncthreads();
  if (tid == 0) __hip_atomic_fetch_add(F.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// Later tiers (non-uniform partitioning, Sec. III-B): partitions of P_t = r B
// samples covering filter taps [o_t, o_t + K_t P_t).  Frame f of the tier is
// input samples [f P_t, (f+1) P_t), complete after block n_f = (f+1) r - 1.
// Its contribution y[f P_t + o_t + i] (i < P_t) is the second half of the
// 2 P_t-point inverse FFT of sum_q sum_p H_{t,l,q,p} X_{t,q}(f - p): the
// tier's delay o_t is realized in the time domain through the output ring.
//
// The 2P_t-point real transforms run as P_t-point complex transforms of
// z[m] = w[2m] + i w[2m+1] (fft_lds.hpp), each factored as P_t = N1 N2 with
// n = n1 + N1 n2 (time) and k = N2 k1 + k2 (frequency):
//   Z[N2 k1 + k2] = sum_n1 W_N1^{n1 k1} W_P^{n1 k2} sum_n2 z[n1 + N1 n2] W_N2^{n2 k2}
// (conjugate twiddles for the inverse).  A pass is a batch of short
// transforms that one 256-thread workgroup runs in LDS; the two passes of a
// transform run in consecutive launches and each pass is spread over several
// workgroups, so no workgroup holds a whole transform and the launch's LDS
// stays small.  Work of frame f, by lag after block n_f (the host's lists):
//   0           K_FFT_A  columns n1: N2-point transforms of the window times
//                        W_P^{n1 k2}, into tfwd[q] (k2-major)
//   1           K_FFT_B  column pairs (k2, N2 - k2): N1-point transforms, the
//                        real-transform split, packed bins into slot f mod K
//   2 .. nmac+1 K_MAC    the frame's multiply-accumulate (tail items)
//   nmac+2      K_FIN_A  column pairs: partial slots summed, the inverse
//                        split, N1-point inverse transforms times
//                        W_P^{-n1 k2}, into tinv[l] (n1-major)
//   nmac+3      K_FIN_B  rows n1: N2-point inverse transforms; the second
//                        half of the samples (overlap-save), scaled by
//                        1/(2P), into the output ring at f P + o_t
// Bin k of the real transform pairs with bin P - k, which lies in column
// N2 - k2 (row N1 - 1 - k1) for k2 > 0 and in column 0 (row N1 - k1) for
// k2 = 0; columns 0 and N2/2 pair with themselves.  A pair item holds both
// columns of each pair: its first np columns are k2 = j np .. j np + np - 1,
// the other np their partners, with column N2/2 in place of column 0's.
// ---------------------------------------------------------------------------
constexpr int kTierBuf = 1024;                 // float2 per LDS buffer of a pass
constexpr int kTierLds = 2 * kTierBuf + 128;   // two buffers and an N-point table (N <= 128)

__host__ __device__ inline int tier_lg1(int logP) { return logP / 2; }
// rows per K_FFT_A / K_FIN_B item (N2-point transforms)
__host__ __device__ inline int tier_rows_per_item(int logP) {
  const int n1 = 1 << tier_lg1(logP), n2 = 1 << (logP - tier_lg1(logP));
  return n1 < kTierBuf / n2 ? n1 : kTierBuf / n2;
}
// column pairs per K_FFT_B / K_FIN_A item (two N1-point transforms each)
__host__ __device__ inline int tier_pairs_per_item(int logP) {
  const int n1 = 1 << tier_lg1(logP), n2 = 1 << (logP - tier_lg1(logP));
  return n2 / 2 < kTierBuf / (2 * n1) ? n2 / 2 : kTierBuf / (2 * n1);
}

// column k2 of local column c (c < 2 np) of pair item j
__device__ __forceinline__ int pair_col(int j, int np, int c, int N2) {
  const int k = j * np + (c < np ? c : c - np);
  if (c < np) return k;
  return k == 0 ? N2 / 2 : N2 - k;
}
// local column holding the partner bins of local column c
__device__ __forceinline__ int pair_partner(int j, int np, int c) {
  if (j * np + (c < np ? c : c - np) == 0) return c;  // columns 0 and N2/2
  return c < np ? c + np : c - np;
}

// Input sample i (< B) of this block for input q as the first tier sees it:
// the microphone minus the previous block's feedback estimate, zero for a
// slot that is not live.  (Fused feedback: the estimate is written in this
// launch by other workgroups, so it is read where every XCD sees it; the
// caller has waited for it.)
__device__ __forceinline__ float block_sample(const KArgs& A, int q, int i) {
  float v = A.in[(int64_t)q * A.B + i];
  if (A.sub != nullptr) {
    const float* p = A.sub + (int64_t)q * A.B + i;
    v -= A.fc_on ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : *p;
  }
  return (A.live != nullptr && A.live[q] == 0) ? 0.f : v;  // a select: NaN stays out
}

template <int G>
__device__ __forceinline__ void tier_fft_a(const KArgs& A, int64_t n, const Item& it, float2* lds) {
  const DevTier& T = A.tier[it.tier];
  const int tid = threadIdx.x, P = T.P;
  const int lg1 = T.lg1, N1 = 1 << lg1, lg2 = T.logP - lg1, N2 = 1 << lg2;
  const int nr = it.w, n10 = it.k0 * nr, q = it.q;
  float2* a = lds;
  float2* b = lds + kTierBuf;
  float2* twn = lds + 2 * kTierBuf;
  for (int j = tid; j < N2; j += kThreads) twn[j] = T.tw[j << lg1];  // W_N2^j = W_P^{j N1}
  if (A.fc_on) fc_wait(A, n);  // the block's samples need c_{n-1}
  // window: the last 2P samples up to the end of this block (its first
  // 2P - B from the history ring)
  const float* hq = A.hist + (int64_t)q * (A.hist_mask + 1);
  const int64_t start = (n - it.lag + 1) * A.B - 2 * (int64_t)P;
  const int cur = 2 * P - A.B;
  auto sample = [&](int i) {
    return i < cur ? hq[(start + i) & A.hist_mask] : block_sample(A, q, i - cur);
  };
  for (int e = tid; e < nr * N2; e += kThreads) {
    const int c = e & (nr - 1), n2 = e / nr;
    const int m = n10 + c + (n2 << lg1);
    a[c * N2 + n2] = make_float2(sample(2 * m), sample(2 * m + 1));
  }
  __syncthreads();
  const float2* z = fft_stockham<false>(a, b, N2, lg2, twn, nr);
  float2* dst = T.tfwd + (int64_t)q * P;
  for (int e = tid; e < nr * N2; e += kThreads) {
    const int c = e & (nr - 1), k2 = e / nr;
    const int n1 = n10 + c;
    dst[k2 * N1 + n1] = cmul(z[c * N2 + k2], T.tw[(n1 * k2) & (P - 1)]);
  }
}

template <int G>
__device__ __forceinline__ void tier_fft_b(const KArgs& A, int64_t n, const Item& it, float2* lds) {
  const DevTier& T = A.tier[it.tier];
  const int tid = threadIdx.x, P = T.P;
  const int lg1 = T.lg1, N1 = 1 << lg1, lg2 = T.logP - lg1, N2 = 1 << lg2;
  const int np = it.w, nc = 2 * np, j = it.k0, q = it.q;
  float2* a = lds;
  float2* b = lds + kTierBuf;
  float2* twn = lds + 2 * kTierBuf;
  for (int i = tid; i < N1; i += kThreads) twn[i] = T.tw[i << lg2];  // W_N1^i
  const float2* src = T.tfwd + (int64_t)q * P;
  for (int e = tid; e < nc * N1; e += kThreads) {
    const int c = e >> lg1, k1 = e & (N1 - 1);
    a[e] = src[pair_col(j, np, c, N2) * N1 + k1];
  }
  __syncthreads();
  const float2* Z = fft_stockham<false>(a, b, N1, lg1, twn, nc);
  // packed bins X[k] = E + W_2P^k O from Z[k] and Z[P - k] (fft_lds.hpp)
  const int64_t f = (n - it.lag + 1) / T.r - 1;
  float2* dst = T.X + ((int64_t)q * T.K + wrap_slot(f, T.K)) * P;
  const float2* tw2 = T.tw + P;
  for (int e = tid; e < nc * N1; e += kThreads) {
    const int c = e & (nc - 1), k1 = e / nc;
    const int k2 = pair_col(j, np, c, N2);
    const int k = (k1 << lg2) + k2;
    const float2 zk = Z[c * N1 + k1];
    float2 x;
    if (k == 0) {
      x = make_float2(zk.x + zk.y, zk.x - zk.y);
    } else {
      const int pk1 = k2 == 0 ? ((N1 - k1) & (N1 - 1)) : N1 - 1 - k1;
      const float2 zm = cconj(Z[pair_partner(j, np, c) * N1 + pk1]);
      const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
      const float2 d = csub(zk, zm);
      const float2 O = make_float2(0.5f * d.y, -0.5f * d.x);  // -i d / 2
      x = cadd(E, cmul(tw2[k], O));
    }
    dst[k] = x;
  }
}

template <int G>
__device__ __forceinline__ void tier_fin_a(const KArgs& A, int64_t n, const Item& it, float2* lds) {
  const DevTier& T = A.tier[it.tier];
  const int tid = threadIdx.x, P = T.P;
  const int lg1 = T.lg1, N1 = 1 << lg1, lg2 = T.logP - lg1, N2 = 1 << lg2;
  const int np = it.w, nc = 2 * np, j = it.k0;
  const Group grp = A.groups[it.group];
  const int gsel = it.q, l = grp.l0 + gsel;
  const int64_t gi = (int64_t)it.tier * A.n_groups_total + it.group;
  const int s0 = A.tier_slot0[gi], ns = A.tier_nslot[gi];
  const int64_t stride = (int64_t)G * P;
  const float2* base = T.partial + (int64_t)s0 * stride + (int64_t)gsel * P;
  float2* a = lds;
  float2* b = lds + kTierBuf;
  float2* twn = lds + 2 * kTierBuf;
  for (int i = tid; i < N1; i += kThreads) twn[i] = T.tw[i << lg2];  // W_N1^i
  // the frame's spectrum in the item's columns: its partial slots, summed in
  // slot order
  for (int e = tid; e < nc * N1; e += kThreads) {
    const int c = e & (nc - 1), k1 = e / nc;
    const int k = (k1 << lg2) + pair_col(j, np, c, N2);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int s = 0; s < ns; ++s) acc = cadd(acc, base[s * stride + k]);
    a[c * N1 + k1] = acc;
  }
  __syncthreads();
  // inverse split (fft_lds.hpp irfft_pre): Z'[k] = E + i O
  const float2* tw2 = T.tw + P;
  for (int e = tid; e < nc * N1; e += kThreads) {
    const int c = e >> lg1, k1 = e & (N1 - 1);
    const int k2 = pair_col(j, np, c, N2);
    const int k = (k1 << lg2) + k2;
    const float2 yk = a[e];
    float2 z;
    if (k == 0) {
      z = make_float2(yk.x + yk.y, yk.x - yk.y);
    } else {
      const int pk1 = k2 == 0 ? ((N1 - k1) & (N1 - 1)) : N1 - 1 - k1;
      const float2 ym = cconj(a[pair_partner(j, np, c) * N1 + pk1]);
      const float2 E = cadd(yk, ym);
      const float2 O = cmul(csub(yk, ym), cconj(tw2[k]));
      z = make_float2(E.x - O.y, E.y + O.x);
    }
    b[e] = z;
  }
  __syncthreads();
  const float2* z = fft_stockham<true>(b, a, N1, lg1, twn, nc);
  float2* dst = T.tinv + (int64_t)l * P;
  for (int e = tid; e < nc * N1; e += kThreads) {
    const int c = e & (nc - 1), n1 = e / nc;
    const int k2 = pair_col(j, np, c, N2);
    dst[n1 * N2 + k2] = cmul(z[c * N1 + n1], cconj(T.tw[(n1 * k2) & (P - 1)]));
  }
}

template <int G>
__device__ __forceinline__ void tier_fin_b(const KArgs& A, int64_t n, const Item& it, float2* lds) {
  const DevTier& T = A.tier[it.tier];
  const int tid = threadIdx.x, P = T.P;
  const int lg1 = T.lg1, lg2 = T.logP - lg1, N2 = 1 << lg2;
  const int nr = it.w, n10 = it.k0 * nr;
  const int l = A.groups[it.group].l0 + it.q;
  float2* a = lds;
  float2* b = lds + kTierBuf;
  float2* twn = lds + 2 * kTierBuf;
  for (int i = tid; i < N2; i += kThreads) twn[i] = T.tw[i << lg1];  // W_N2^i
  const float2* src = T.tinv + (int64_t)l * P + (int64_t)n10 * N2;
  for (int e = tid; e < nr * N2; e += kThreads) a[e] = src[e];
  __syncthreads();
  const float2* z = fft_stockham<true>(a, b, N2, lg2, twn, nr);
  // complex samples m = n1 + N1 n2 >= P/2 (n2 >= N2/2): output samples
  // 2m - P, 2m - P + 1 of the frame
  const int64_t f = (n - it.lag + 1) / T.r - 1;
  const int64_t y0 = f * (int64_t)P + T.offset;
  float* ring = T.oring + (int64_t)l * (A.ring_mask + 1);
  const float scale = 1.0f / (float)(2 * P);
  const int h2 = N2 >> 1;
  for (int e = tid; e < nr * h2; e += kThreads) {
    const int c = e & (nr - 1), h = e / nr;
    const float2 v = z[c * N2 + h2 + h];
    const int64_t i0 = 2 * (int64_t)(n10 + c + (h << lg1));
    ring[(y0 + i0) & A.ring_mask] = v.x * scale;
    ring[(y0 + i0 + 1) & A.ring_mask] = v.y * scale;
  }
}

template <int G>
__device__ __forceinline__ void tier_pass(const KArgs& A, int64_t n, const Item& it, float2* lds) {
  switch (it.kind) {
    case K_FFT_A: tier_fft_a<G>(A, n, it, lds); break;
    case K_FFT_B: tier_fft_b<G>(A, n, it, lds); break;
    case K_FIN_A: tier_fin_a<G>(A, n, it, lds); break;
    case K_FIN_B: tier_fin_b<G>(A, n, it, lds); break;
    default: break;
  }
}

template <typename HT, int G, bool NT>
__global__ __launch_bounds__(kThreads) void k_block(const KArgs A) {
  extern __shared__ float2 lds[];
  // the block index: from the launch, or (graph replay) the device counter
  // plus this launch's place in the graph
  // Kernel-argument fields are read where first used, after the branch
  // before them, one scalar round trip after another; an empty asm that
  // takes the dispatch's fields as operands makes them one batch up front.
  {
    const void* nb = A.n_base;
    const int64_t n0 = A.n;
    const int fc = A.fc_on, fs = A.fc.head_slots, fh = A.fc.n_heads, hs = A.head_slots, nh = A.n_head,
              ts = A.tier_slots, np = A.n_phase, mi = A.max_items, tw = A.tails_wait;
    const void* it = A.items;
    const void* gr = A.groups;
    asm volatile("" ::"s"(nb), "s"(n0), "s"(fc), "s"(fs), "s"(fh), "s"(hs), "s"(nh), "s"(ts), "s"(np), "s"(mi),
                 "s"(tw), "s"(it), "s"(gr));
  }
  const int64_t n = A.n_base != nullptr ? *A.n_base + A.n : A.n;
  int b = blockIdx.x;
  if (A.fc_on) {  // grid: feedback heads | heads | transforms | tails | feedback tails
    if (b < A.fc.head_slots) {
      if (b < A.fc.n_heads) fc_head_work<HT, G>(A, n, b, lds);
      return;
    }
    b -= A.fc.head_slots;
  }
  if (b < A.head_slots) {
    if (b < A.n_head) {  // head b: output b, in group b / G
      const Group g0 = A.groups[b / G];
      Group hg = g0;
      hg.l0 = b;
      hg.nl = 1;
      head_work<HT, G>(A, n, hg, b - g0.l0, lds);
    }
    return;
  }
  // later tiers' transform passes of this phase, then the tails (uniform
  // partitions: one phase, no 64-bit division)
  const int phase = A.n_phase == 1 ? 0 : (int)(n % A.n_phase);
  b -= A.head_slots;
  if (b < A.tier_slots) {
    if (b < A.tier_count[phase])
      tier_pass<G>(A, n, A.tier_items[(int64_t)phase * A.max_tier_items + b], lds);
    return;
  }
  const int i = b - A.tier_slots;
  // rta_process: the heads of this launch are the block's latency path, and
  // they run slower on compute units that streaming tails share; the
  // multiply-accumulate (for the next block) waits until they are done.  A
  // bounded wait that gives up only costs time: the tails read nothing the
  // heads write.
  if (A.tails_wait) {
    if (threadIdx.x == 0) {
      const unsigned int target = (unsigned int)((n + 1) * A.n_head);
      for (int it = 0; it < 512; ++it) {  // about 0.2 ms at most
        if ((int)(__hip_atomic_load(A.heads_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) >= 0)
          break;
        __builtin_amdgcn_s_sleep(16);
      }
    }
    __syncthreads();
  }
  if (A.fc_on && i >= A.fc.tail0) {  // feedback terms p >= 2 for c_n
    const int j = i - A.fc.tail0;
    if (j >= A.fc.n_items) return;
    const Item it = A.fc.items[j];
    if (it.kind == K_NOP) return;
    DevTier T = A.fc.T;
    T.partial += (n & 1) * (int64_t)T.nslots * G * T.P;
    mac_item<HT, G, NT>(T, it, n, lds);
    return;
  }
  // (the tail part of the grid is at most max_items long, and a phase's
  // list is padded to max_items with K_NOP).  The first tier's fields are
  // read before the item arrives: most items are first-tier ones.
  DevTier T = A.tier[0];
  asm volatile("" ::"s"(T.H), "s"(T.X), "s"(T.partial), "s"(T.K), "s"(T.P), "s"(T.nslots));
  const Item it = A.items[(int64_t)phase * A.max_items + i];
  if (it.kind == K_NOP) return;
  if (it.tier != 0) T = A.tier[it.tier];
  int64_t frame;
  if (it.tier == 0) {
    frame = n + 1;  // first-tier tails prepare the next block
    T.partial += (frame & 1) * (int64_t)T.nslots * G * T.P;
  } else {
    // later tier: the frame whose input completed in block n - lag
    frame = (n - it.lag + 1) / T.r - 1;
  }
  mac_item<HT, G, NT>(T, it, frame, lds);
}

// Graph replay's device block counter: set to v (add = 0), or advanced by v
// (add = 1) by the graph's last node.
__global__ void k_counter(int64_t* ctr, int64_t v, int32_t add) {
  if (threadIdx.x == 0) *ctr = add ? *ctr + v : v;
}

// Dense copy of partitions 0 and 1 of every pair for the heads:
// H01[l][q][r][P] = row r of pair (l, q), or zeros if the pair has no row r.
template <typename HT>
__global__ __launch_bounds__(kThreads) void k_gather_head_rows(const HT* H, const int64_t* pair_row,
                                                              const int32_t* pair_K, int P,
                                                              int n_pairs, HT* H01) {
  const int pr = blockIdx.x;  // pair * 2 + r
  if (pr >= 2 * n_pairs) return;
  const int pair = pr >> 1, r = pr & 1;
  const int64_t row = pair_row[pair];
  const bool has = row >= 0 && r < pair_K[pair];
  for (int k = threadIdx.x; k < P; k += kThreads) {
    HT v{};
    if (has) v = H[(row + r) * (int64_t)P + k];
    H01[(int64_t)pr * P + k] = v;
  }
}

// ---------------------------------------------------------------------------
// Streaming-read probe (measurement aid): workgroup w reads its contiguous
// chunk of n16 16-byte vectors with the same non-temporal loads as k_mac,
// kUnroll vectors in flight per thread, and writes one float so the loads
// are not removed.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_read_probe(const f32x4* __restrict__ buf,
                                                        int64_t n16, float* sink) {
  __shared__ float red[kThreads];
  const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min(n16, b0 + per);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  int64_t i = b0 + threadIdx.x;
  for (; i + (kUnroll - 1) * kThreads < b1; i += kUnroll * kThreads) {
    f32x4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(buf + i + u * kThreads);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += v[u];
  }
  for (; i < b1; i += kThreads) acc += __builtin_nontemporal_load(buf + i);
  red[threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int k = 0; k < kThreads; ++k) t += red[k];
    sink[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Filter spectra (create time): one workgroup per partition row.  Row r takes
// taps [src, src+len) (len <= P), zero-pads to 2P (sub-filter followed by P
// zeros, Sec. IV), real-FFTs and stores P packed bins.
// ---------------------------------------------------------------------------
struct SpecRow {
  int64_t src;   // offset into the staged taps
  int64_t dst;   // destination row
  int32_t len;   // valid taps (<= P)
  int32_t pad;
};

__device__ __forceinline__ void store_bin(float2* H, int64_t i, float2 v, int*) { H[i] = v; }

__device__ __forceinline__ void store_bin(f16c_t* H, int64_t i, float2 v, int* range) {
  if (fabsf(v.x) > 65504.f || fabsf(v.y) > 65504.f || v.x != v.x || v.y != v.y) atomicOr(range, 1);
  const _Float16 re = (_Float16)v.x;  // round to nearest even
  const _Float16 im = (_Float16)v.y;
  H[i].bits = (uint32_t)__builtin_bit_cast(uint16_t, re) |
              ((uint32_t)__builtin_bit_cast(uint16_t, im) << 16);
}

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void store_bin(bf16c_t* H, int64_t i, float2 v, int*) {
  H[i].bits = bf16_rne(v.x) | (bf16_rne(v.y) << 16);
}

template <typename HT>
__global__ __launch_bounds__(kThreads) void k_spectra(const float* taps, const SpecRow* rows,
                                                      HT* H, int P, int logP, int r3,
                                                      const float2* tw, int* range) {
  extern __shared__ float2 lds[];
  float2* a = lds;
  float2* b = lds + P;
  const SpecRow row = rows[blockIdx.x];
  for (int m = threadIdx.x; m < P; m += kThreads) {
    const int i0 = 2 * m, i1 = 2 * m + 1;
    a[m] = make_float2(i0 < row.len ? taps[row.src + i0] : 0.f,
                       i1 < row.len ? taps[row.src + i1] : 0.f);
  }
  __syncthreads();
  float2* z = fft_any<false>(a, b, P, logP, r3, tw);
  float2* x = (z == a) ? b : a;
  rfft_post(z, x, P, tw + P);
  for (int k = threadIdx.x; k < P; k += kThreads) store_bin(H, row.dst * P + k, x[k], range);
}

}  // namespace rta
