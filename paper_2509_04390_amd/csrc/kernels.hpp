// kernels.hpp -- gfx950 kernels of the partitioned convolution.
//
// Two launches per audio block, ordered on one stream.
//
// k_mac: workgroup i runs work item i of the block's phase list.  Items of
// kind MAC0 cover the uniform first tier (partition = block, Sec. IV): an
// item owns a group of G outputs, one input q, a partition range [p0, p1) and
// a slice of bins, and computes
//     Y_l[k] += sum_{p in [p0,p1)} H_{l,q,p}[k] * X_q[(n - p) mod K][k]
// (Sec. IV step 2, frequency-domain delay line as a ring with a head index).
// Items whose range starts at p = 0 transform the current input window
// themselves (Sec. IV step 1: last 2B samples, real FFT), so no launch is
// spent on the forward transform; one of them stores that spectrum into the
// ring slot n mod K for later blocks.  Each item writes its partial sums to
// its own slot.
//
// k_final: one workgroup per output group adds the group's slots in a fixed
// order, runs the inverse real FFT and keeps the second half of the 2B
// samples (overlap-save, Sec. IV step 3).
//
// The block index lives in device memory and k_final advances it, so
// identical launches (and graph replays) process successive blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace rta {

constexpr int kThreads = 256;
constexpr int kMaxTiers = 8;
constexpr int kUnroll = 4;

enum ItemKind : int32_t { K_MAC0 = 0, K_MAC = 1, K_FFT = 2, K_NOP = 3 };
enum ItemFlag : int32_t { F_WRITE_X = 1, F_WRITE_HIST = 2, F_FINAL = 4 };

struct Item {          // one workgroup's work in one block (48 bytes)
  int32_t kind;        // ItemKind
  int32_t flags;       // ItemFlag bits
  int32_t tier;
  int32_t group;       // reduction group (outputs l0 .. l0+nl-1)
  int32_t q;           // input channel
  int32_t p0, p1;      // partition range
  int32_t k0;          // first bin of the slice
  int32_t slot;        // partial-sum slot (tier-local)
  int32_t target;      // items of this group launched in this block
  int32_t lag;         // tiers >= 1: blocks since the frame's input completed
  int32_t pad;
};

struct Group {         // outputs reduced together (16 bytes)
  int32_t l0, nl;      // first output, outputs in the group (<= G)
  int32_t slot0, nslot;
};

struct DevTier {
  const void* H;             // spectra rows [row][P] of the storage type
  const int64_t* pair_row;   // [L*Q] first row of pair (l,q), -1 = no path
  const int32_t* pair_K;     // [L*Q] partitions of pair (l,q)
  float2* X;                 // FDL ring [Q][K][P]
  float2* partial;           // [slots][G][P]
  const float2* tw;          // W_P^j (j<P) then W_2P^k (k<P)
  float* oring;              // tiers >= 1: output ring [L][R]
  int64_t offset;            // first filter tap of the tier
  int32_t P, logP, K, pad;
};

struct DevState {
  int64_t block;             // index of the next block to process
  uint32_t arrive;           // workgroups of the current launch that read it
  uint32_t pad;
};

struct KArgs {
  DevTier tier[kMaxTiers];
  const Item* items;         // [n_phase][max_items]
  const int32_t* phase_count;
  const Group* groups;
  DevState* state;
  float* hist;               // input history [Q][hist_len]
  const float* in;           // [Q][B]
  float* out;                // [L][B]
  int64_t hist_mask;         // hist_len - 1
  int64_t ring_mask;         // output ring length - 1
  int32_t B, Q, L, n_tiers;
  int32_t n_phase, max_items;
};

// ---------------------------------------------------------------------------
// Filter-spectrum element loads: C complex bins per 16-byte vector.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct f16c_t { uint32_t bits; };   // packed (re, im) FP16 pair
struct bf16c_t { uint32_t bits; };  // packed (re, im) BF16 pair

template <typename HT> struct HVec;

template <> struct HVec<float2> {
  static constexpr int C = 2;
  static __device__ __forceinline__ void load(const float2* p, float2 (&h)[C]) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    h[0] = make_float2(v.x, v.y);
    h[1] = make_float2(v.z, v.w);
  }
};

template <> struct HVec<f16c_t> {
  static constexpr int C = 4;
  static __device__ __forceinline__ void load(const f16c_t* p, float2 (&h)[C]) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    // Each 32-bit word is one (re, im) pair.  The halves are taken apart as
    // scalars: a vector bit_cast of v[j] here makes the compiler drop three
    // of the four words of the load.
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t w = v[j];
      const _Float16 re = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
      const _Float16 im = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
      h[j] = make_float2((float)re, (float)im);
    }
  }
};

template <> struct HVec<bf16c_t> {
  static constexpr int C = 4;
  static __device__ __forceinline__ void load(const bf16c_t* p, float2 (&h)[C]) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
#pragma unroll
    for (int j = 0; j < 4; ++j)
      h[j] = make_float2(__uint_as_float(v[j] << 16), __uint_as_float(v[j] & 0xffff0000u));
  }
};

template <int C>
__device__ __forceinline__ void load_x(const float2* p, float2 (&x)[C]) {
#pragma unroll
  for (int j = 0; j < C; j += 2) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(p + j);
    x[j] = make_float2(v.x, v.y);
    x[j + 1] = make_float2(v.z, v.w);
  }
}

__device__ __forceinline__ int wrap_slot(int64_t v, int K) {
  int s = (int)(v % K);
  return s < 0 ? s + K : s;
}

// ---------------------------------------------------------------------------
// Multiply-accumulate of one item's partitions into its partial-sum slot.
// x0 (LDS) holds the fresh spectrum of the current frame, used for p == 0.
// `frame` is the frame whose delay-line head is slot frame mod K.
// ---------------------------------------------------------------------------
template <typename HT, int G>
__device__ void mac_item(const KArgs& A, const DevTier& T, const Item& it,
                         const Group& grp, int64_t frame, const float2* x0,
                         float2* red) {
  constexpr int C = HVec<HT>::C;
  const int P = T.P;
  const int W = P < kThreads * C ? P : kThreads * C;  // bins per item slice
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
    pend[g] = 0;
    hb[g] = Hbase;
    if (g < grp.nl) {
      const int pair = (grp.l0 + g) * A.Q + q;
      const int64_t row = T.pair_row[pair];
      if (row >= 0) {
        pend[g] = min(it.p1, T.pair_K[pair]);
        hb[g] = Hbase + row * (int64_t)P + kb;
      }
    }
  }

  float acc[G][C][4];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < C; ++j) acc[g][j][0] = acc[g][j][1] = acc[g][j][2] = acc[g][j][3] = 0.f;

  auto mac = [&](int g, const float2 (&h)[C], const float2 (&x)[C]) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      acc[g][j][0] += h[j].x * x[j].x;   // Re H Re X
      acc[g][j][1] += h[j].y * x[j].y;   // Im H Im X
      acc[g][j][2] += h[j].x * x[j].y;   // Re H Im X
      acc[g][j][3] += h[j].y * x[j].x;   // Im H Re X
    }
  };

  int p = it.p0 + s;
  if (x0 != nullptr && p == 0) {
    float2 x[C];
#pragma unroll
    for (int j = 0; j < C; ++j) x[j] = x0[kb + j];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (0 < pend[g]) {
        float2 h[C];
        HVec<HT>::load(hb[g], h);
        mac(g, h, x);
      }
    }
    p += RP;
  }

  const int K = T.K;
  const float2* Xq = T.X + (int64_t)q * K * P + kb;
  const int step = RP % K;
  int slot = wrap_slot(frame - p, K);
  for (; p < it.p1; p += RP * kUnroll) {
    float2 xv[kUnroll][C];
    float2 hv[kUnroll][G][C];
    int sl = slot;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int pu = p + u * RP;
      if (pu < it.p1) {
        load_x<C>(Xq + (int64_t)sl * P, xv[u]);
      } else {
#pragma unroll
        for (int j = 0; j < C; ++j) xv[u][j] = make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (pu < pend[g]) {
          HVec<HT>::load(hb[g] + (int64_t)pu * P, hv[u][g]);
        } else {
#pragma unroll
          for (int j = 0; j < C; ++j) hv[u][g][j] = make_float2(0.f, 0.f);
        }
      }
      sl -= step;
      if (sl < 0) sl += K;
    }
    slot = sl;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int g = 0; g < G; ++g) mac(g, hv[u][g], xv[u]);
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

  float2* part = T.partial + (int64_t)it.slot * G * P;
  if (RP == 1) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < C; ++j) part[(int64_t)g * P + kb + j] = res[g][j];
    return;
  }
  __syncthreads();  // x0 may share LDS with `red`
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < C; ++j) red[(s * G + g) * W + r * C + j] = res[g][j];
  __syncthreads();
  for (int e = tid; e < G * W; e += kThreads) {
    const int g = e / W, b = e - g * W;
    float2 sum = red[g * W + b];
    for (int s2 = 1; s2 < RP; ++s2) sum = cadd(sum, red[(s2 * G + g) * W + b]);
    part[(int64_t)g * P + it.k0 + b] = sum;
  }
}

// Real FFT of the window [x_{n-1}, x_n] of input q (2B samples, first tier).
// Returns the LDS buffer holding the packed spectrum.
__device__ float2* first_tier_spectrum(const KArgs& A, const DevTier& T, int q,
                                       int64_t n, float2* a, float2* b) {
  const int P = T.P;  // == B
  const float* hq = A.hist + (int64_t)q * (A.hist_mask + 1);
  const float* iq = A.in + (int64_t)q * A.B;
  for (int m = threadIdx.x; m < P; m += kThreads) {
    float w[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = 2 * m + e;
      w[e] = i < P ? hq[((n - 1) * A.B + i) & A.hist_mask] : iq[i - P];
    }
    a[m] = make_float2(w[0], w[1]);
  }
  __syncthreads();
  float2* z = fft_stockham<false>(a, b, P, T.logP, T.tw);
  float2* x = (z == a) ? b : a;
  rfft_post(z, x, P, T.tw + P);
  return x;
}

// Sum the group's partial slots for output g of the group into LDS `y`.
template <int G>
__device__ void reduce_slots(const DevTier& T, const Group& grp, int g, float2* y) {
  const int P = T.P;
  const float2* base = T.partial + (int64_t)grp.slot0 * G * P + (int64_t)g * P;
  for (int k = threadIdx.x; k < P; k += kThreads) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int sl = 0; sl < grp.nslot; ++sl) acc = cadd(acc, base[(int64_t)sl * G * P + k]);
    y[k] = acc;
  }
  __syncthreads();
}

// Last workgroup of a first-tier group: reduce, inverse real FFT, keep the
// last B samples, add the later tiers' contributions from their output rings
// and emit the block.
template <int G>
__device__ void first_tier_final(const KArgs& A, const DevTier& T, const Group& grp,
                                 int64_t n, float2* a, float2* b) {
  const int P = T.P;  // == B
  const float scale = 1.0f / (float)(2 * P);
  for (int g = 0; g < grp.nl; ++g) {
    const int l = grp.l0 + g;
    reduce_slots<G>(T, grp, g, a);
    irfft_pre(a, b, P, T.tw + P);
    float2* z = fft_stockham<true>(b, a, P, T.logP, T.tw);
    float* o = A.out + (int64_t)l * A.B;
    for (int m = (P >> 1) + threadIdx.x; m < P; m += kThreads) {
      const float2 v = z[m];
      const int i = 2 * (m - (P >> 1));
      float y0 = v.x * scale, y1 = v.y * scale;
      for (int t = 1; t < A.n_tiers; ++t) {
        float* ring = A.tier[t].oring + (int64_t)l * (A.ring_mask + 1);
        const int64_t s0 = (n * A.B + i) & A.ring_mask;
        const int64_t s1 = (n * A.B + i + 1) & A.ring_mask;
        y0 += ring[s0];
        y1 += ring[s1];
        ring[s0] = 0.f;
        ring[s1] = 0.f;
      }
      o[i] = y0;
      o[i + 1] = y1;
    }
    __syncthreads();
  }
}

template <typename HT, int G>
__global__ __launch_bounds__(kThreads) void k_mac(const KArgs A) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int64_t n = A.state->block;  // advanced only by k_final of the previous block
  const int phase = (int)(n % A.n_phase);
  if ((int)blockIdx.x >= A.phase_count[phase]) return;
  const Item it = A.items[(int64_t)phase * A.max_items + blockIdx.x];
  if (it.kind == K_NOP) return;

  const DevTier& T = A.tier[it.tier];
  const Group grp = A.groups[it.group];
  float2* bufA = lds;
  float2* bufB = lds + T.P;

  if (it.kind == K_MAC0) {
    const float2* x0 = nullptr;
    if (it.p0 == 0) {
      float2* xs = first_tier_spectrum(A, T, it.q, n, bufA, bufB);
      constexpr int C = HVec<HT>::C;
      const int W = T.P < kThreads * C ? T.P : kThreads * C;
      if (it.flags & F_WRITE_X) {
        float2* dst = T.X + ((int64_t)it.q * T.K + wrap_slot(n, T.K)) * T.P;
        for (int k = it.k0 + tid; k < it.k0 + W; k += kThreads) dst[k] = xs[k];
      }
      if (it.flags & F_WRITE_HIST) {
        float* hq = A.hist + (int64_t)it.q * (A.hist_mask + 1);
        const float* iq = A.in + (int64_t)it.q * A.B;
        for (int i = tid; i < A.B; i += kThreads) hq[(n * A.B + i) & A.hist_mask] = iq[i];
      }
      x0 = xs;
    }
    mac_item<HT, G>(A, T, it, grp, n, x0, lds);
  }
}

// One workgroup per output group: reduce the group's partial slots, inverse
// FFT, overlap-save output.  Runs after k_mac of the same block on the same
// stream, so every partial is visible without in-kernel fences.  The last
// workgroup to read the block index advances it for the next block.
template <int G>
__global__ __launch_bounds__(kThreads) void k_final(const KArgs A) {
  extern __shared__ float2 lds[];
  __shared__ int64_t sh_n;
  if (threadIdx.x == 0) sh_n = A.state->block;
  __syncthreads();
  const int64_t n = sh_n;
  if (threadIdx.x == 0) {
    const uint32_t old = __hip_atomic_fetch_add(&A.state->arrive, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == gridDim.x - 1) {  // every workgroup has read n
      A.state->arrive = 0;
      A.state->block = n + 1;
    }
  }
  const DevTier& T = A.tier[0];
  const Group grp = A.groups[blockIdx.x];
  first_tier_final<G>(A, T, grp, n, lds, lds + T.P);
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
                                                      HT* H, int P, int logP,
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
  float2* z = fft_stockham<false>(a, b, P, logP, tw);
  float2* x = (z == a) ? b : a;
  rfft_post(z, x, P, tw + P);
  for (int k = threadIdx.x; k < P; k += kThreads) store_bin(H, row.dst * P + k, x[k], range);
}

}  // namespace rta
