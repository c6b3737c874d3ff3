// fft_lds.hpp -- workgroup-cooperative FFTs staged in LDS (gfx950, wave64).
//
// Complex FFT: Stockham autosort, radix 4 with one radix-2 stage when log2 N
// is odd, ping-ponging between two LDS buffers so the result comes out in
// natural order without a bit-reversal pass.  Stage with radix R and
// sub-transform length Ns (Ns = 1, R, R^2, ...): element j of the stage
// (j < N/R, k = j mod Ns) reads a[j + r N/R], multiplies by W_{R Ns}^{r k},
// does an R-point DFT and writes b[(j - k) R + k + r Ns].
//
// Real FFT of 2P samples via one P-point complex FFT (the usual even/odd
// split): z[m] = w[2m] + i w[2m+1], Z = FFT_P(z), then
//   E = (Z[k] + conj Z[P-k]) / 2,  O = -i (Z[k] - conj Z[P-k]) / 2,
//   X[k] = E + W_2P^k O,  X[P-k] = conj(E - W_2P^k O).
// The P bins are stored "packed": bin 0 carries the two real values DC and
// Nyquist as (X[0], X[P]); bins 1..P-1 are the ordinary complex bins.  The
// inverse undoes the split and leaves the 1/(2P) factor to the caller.
//
// Twiddles are host-generated in FP64 and rounded once to FP32; a tier's
// table holds W_P^j (j < P) followed by W_2P^k (k < P), W_N = exp(-2 pi i/N).
#pragma once

#include <hip/hip_runtime.h>

namespace rta {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Batched complex FFT: nb transforms of length N = 2^logN stored back to back
// in LDS buffer `a` ([nb][N]); `b` is LDS scratch of the same size.  INV
// selects exp(+2 pi i/N) twiddles (unnormalized).  Every thread of the
// workgroup must call it; it returns the buffer that holds the results and
// ends with a barrier.
template <bool INV>
__device__ float2* fft_stockham(float2* a, float2* b, int N, int logN,
                                const float2* __restrict__ tw, int nb = 1) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int Ns = 1, rem = logN;
  while (rem > 0) {
    if (rem >= 2) {
      const int quarter = N >> 2;
      const int ts = N / (Ns << 2);
      const int total = nb * quarter;
      for (int w = tid; w < total; w += nt) {
        const int bb = w >> (logN - 2), j = w & (quarter - 1);
        const float2* ab = a + bb * N;
        float2* bbuf = b + bb * N;
        const int k = j & (Ns - 1);
        float2 v0 = ab[j], v1 = ab[j + quarter], v2 = ab[j + 2 * quarter], v3 = ab[j + 3 * quarter];
        if (Ns > 1) {
          float2 w1 = tw[k * ts], w2 = tw[2 * k * ts], w3 = tw[3 * k * ts];
          if (INV) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
          v1 = cmul(v1, w1); v2 = cmul(v2, w2); v3 = cmul(v3, w3);
        }
        const float2 s02 = cadd(v0, v2), d02 = csub(v0, v2);
        const float2 s13 = cadd(v1, v3), d13 = csub(v1, v3);
        // forward: -i * d13 ; inverse: +i * d13
        const float2 jd = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
        const int base = ((j - k) << 2) + k;
        bbuf[base] = cadd(s02, s13);
        bbuf[base + Ns] = cadd(d02, jd);
        bbuf[base + 2 * Ns] = csub(s02, s13);
        bbuf[base + 3 * Ns] = csub(d02, jd);
      }
      Ns <<= 2;
      rem -= 2;
    } else {
      const int half = N >> 1;
      const int ts = N / (Ns << 1);
      const int total = nb * half;
      for (int w = tid; w < total; w += nt) {
        const int bb = w >> (logN - 1), j = w & (half - 1);
        const float2* ab = a + bb * N;
        float2* bbuf = b + bb * N;
        const int k = j & (Ns - 1);
        float2 v0 = ab[j], v1 = ab[j + half];
        if (Ns > 1) {
          float2 w = tw[k * ts];
          if (INV) w.y = -w.y;
          v1 = cmul(v1, w);
        }
        const int base = ((j - k) << 1) + k;
        bbuf[base] = cadd(v0, v1);
        bbuf[base + Ns] = csub(v0, v1);
      }
      Ns <<= 1;
      rem -= 1;
    }
    __syncthreads();
    float2* t = a; a = b; b = t;
  }
  return a;
}

// Batched complex FFT of length N = 3 * 2^m (the 3B-point real transforms of
// the n_f = 3 n_x variant run as N = 3B/2-point complex ones): a radix-3
// Stockham stage first (sub-transform length 1, no twiddles), then radix-4
// stages and a last radix-2 stage over the 2^m factor, with the same stage
// rule as fft_stockham and twiddles W_N^j from `tw` (N entries).  Index
// arithmetic divides by N / R and takes k = j mod Ns with Ns = 3 * 4^i, so
// it is kept apart from the power-of-two routine.  Every thread of the
// workgroup must call it; returns the buffer with the results, ends with a
// barrier.
template <bool INV>
__device__ float2* fft_stockham3(float2* a, float2* b, int N, int m,
                                 const float2* __restrict__ tw, int nb = 1) {
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr float kS3 = 0.86602540378443864676f;  // sqrt(3) / 2
  {
    const int third = N / 3;
    for (int w = tid; w < nb * third; w += nt) {
      const int bb = w / third, j = w - bb * third;
      const float2* ab = a + bb * N;
      float2* bbuf = b + bb * N;
      const float2 v0 = ab[j], v1 = ab[j + third], v2 = ab[j + 2 * third];
      const float2 t1 = cadd(v1, v2);
      const float2 t2 = make_float2(v0.x - 0.5f * t1.x, v0.y - 0.5f * t1.y);
      const float2 d = csub(v1, v2);
      // forward: y1 = t2 - i s d, y2 = t2 + i s d (s = sqrt(3)/2); inverse swaps
      const float2 isd = INV ? make_float2(-kS3 * d.y, kS3 * d.x) : make_float2(kS3 * d.y, -kS3 * d.x);
      bbuf[3 * j] = cadd(v0, t1);
      bbuf[3 * j + 1] = cadd(t2, isd);
      bbuf[3 * j + 2] = csub(t2, isd);
    }
    __syncthreads();
    float2* t = a; a = b; b = t;
  }
  int Ns = 3, rem = m;
  while (rem > 0) {
    const int R = rem >= 2 ? 4 : 2;
    const int per = N / R;
    const int ts = N / (Ns * R);
    for (int w = tid; w < nb * per; w += nt) {
      const int bb = w / per, j = w - bb * per;
      const float2* ab = a + bb * N;
      float2* bbuf = b + bb * N;
      const int k = j % Ns;
      const int base = (j - k) * R + k;
      if (R == 4) {
        float2 v0 = ab[j], v1 = ab[j + per], v2 = ab[j + 2 * per], v3 = ab[j + 3 * per];
        float2 w1 = tw[k * ts], w2 = tw[2 * k * ts], w3 = tw[3 * k * ts];
        if (INV) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
        v1 = cmul(v1, w1); v2 = cmul(v2, w2); v3 = cmul(v3, w3);
        const float2 s02 = cadd(v0, v2), d02 = csub(v0, v2);
        const float2 s13 = cadd(v1, v3), d13 = csub(v1, v3);
        const float2 jd = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
        bbuf[base] = cadd(s02, s13);
        bbuf[base + Ns] = cadd(d02, jd);
        bbuf[base + 2 * Ns] = csub(s02, s13);
        bbuf[base + 3 * Ns] = csub(d02, jd);
      } else {
        float2 v0 = ab[j], v1 = ab[j + per];
        float2 w1 = tw[k * ts];
        if (INV) w1.y = -w1.y;
        v1 = cmul(v1, w1);
        bbuf[base] = cadd(v0, v1);
        bbuf[base + Ns] = csub(v0, v1);
      }
    }
    __syncthreads();
    float2* t = a; a = b; b = t;
    Ns *= R;
    rem -= R == 4 ? 2 : 1;
  }
  return a;
}

// Bit reversal of s over log2(V) bits, V in {1, 2, 4, 8}.
template <int V>
__device__ __forceinline__ constexpr int brev_small(int s) {
  return V == 1 ? 0 : V == 2 ? s : V == 4 ? ((s & 1) << 1) | (s >> 1)
                                        : ((s & 1) << 2) | (s & 2) | (s >> 2);
}

// v of lane (lane ^ H) for a butterfly partner at distance H: quad
// permutations (DPP, a VALU operand modifier) for 1 and 2, the LDS
// crossbar's swizzle (bit mode, xor mask; no address operand) for 4 to 16,
// the gfx950 half-wave swap (VALU) for 32.
template <int H>
__device__ __forceinline__ float lane_xor(float v, int lane) {
  const int i = __float_as_int(v);
  int o;
  if constexpr (H == 1)
    o = __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
  else if constexpr (H == 2)
    o = __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
  else if constexpr (H < 32)
    o = __builtin_amdgcn_ds_swizzle(i, 0x1F | (H << 10));  // and 0x1f, or 0, xor H
  else {
    // half-wave swap of v with itself: the partner values are in the second
    // result for lanes below 32, in the first for the others
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)i, (unsigned)i, false, false);
    o = (int)((lane & 32) ? r[0] : r[1]);
  }
  return __int_as_float(o);
}
// One radix-2 DIF stage across lanes at distance H for V registers per lane.
template <bool INV, int V, int H>
__device__ __forceinline__ void wave_stage(float2 (&r)[V], int N, const float2* __restrict__ tw, int lane) {
  const bool hi = (lane & H) != 0;
  float2 w = tw[(lane & (H - 1)) * (N / (2 * H))];
  if (INV) w.y = -w.y;
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const float2 p = make_float2(lane_xor<H>(r[s].x, lane), lane_xor<H>(r[s].y, lane));
    r[s] = hi ? cmul(csub(p, r[s]), w) : cadd(r[s], p);
  }
}

// One N = 64 V-point transform (V in {1, 2}; brev_small and the in-lane
// stage also cover 4 and 8) by one wavefront, without barriers: lane i
// holds x[64 v + i] (v < V) in registers, with n = 64 v + i and
// k = k1 + V k2 the transform factors as
//   X[k1 + V k2] = sum_i W_64^{i k2} W_N^{i k1} sum_v x[64 v + i] W_V^{v k1}:
// a V-point DIF in each lane's registers, the twiddles W_N^{i k1}, then a
// 64-point radix-2 DIF across the lanes whose butterfly partners are
// exchanged across lanes (distance 32, 16, ..., 1; lane_xor).  Lane i then
// holds k2 = bitrev6(i) and register s holds k1 = bitrev(s); each value is written
// to its natural place in `dst`.  `tw` = W_N^j (j < N); INV conjugates.
template <bool INV, int V>
__device__ __forceinline__ void fft_wave_one(const float2* __restrict__ src, float2* __restrict__ dst,
                                             int N, const float2* __restrict__ tw, int lane) {
  auto twid = [&](int j) {
    float2 w = tw[j];
    if (INV) w.y = -w.y;
    return w;
  };
  float2 r[V];
#pragma unroll
  for (int v = 0; v < V; ++v) r[v] = src[64 * v + lane];
#pragma unroll
  for (int h = V / 2; h >= 1; h /= 2) {
#pragma unroll
    for (int blk = 0; blk < V; blk += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const float2 p = r[blk + j], q = r[blk + j + h];
        r[blk + j] = cadd(p, q);
        r[blk + j + h] = j == 0 ? csub(p, q) : cmul(csub(p, q), twid(j * (V / (2 * h)) * 64));
      }
    }
  }
#pragma unroll
  for (int s = 1; s < V; ++s) r[s] = cmul(r[s], twid(lane * brev_small<V>(s)));
  wave_stage<INV, V, 32>(r, N, tw, lane);
  wave_stage<INV, V, 16>(r, N, tw, lane);
  wave_stage<INV, V, 8>(r, N, tw, lane);
  wave_stage<INV, V, 4>(r, N, tw, lane);
  wave_stage<INV, V, 2>(r, N, tw, lane);
  wave_stage<INV, V, 1>(r, N, tw, lane);
  const int k2 = (int)(__brev((unsigned int)lane) >> 26);
#pragma unroll
  for (int s = 0; s < V; ++s) dst[brev_small<V>(s) + V * k2] = r[s];
}

// Batched complex FFT of length N in {64, 128}: transform t is run
// by wavefront t mod (blockDim.x / 64), reading `a` and writing `b` (LDS,
// [nb][N] each); the stages inside a transform need no workgroup barrier.
// Returns `b`; ends with a barrier.
template <bool INV>
__device__ __forceinline__ float2* fft_wave(float2* a, float2* b, int N, const float2* __restrict__ tw, int nb) {
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int t = threadIdx.x >> 6; t < nb; t += nw) {
    const float2* src = a + t * N;
    float2* dst = b + t * N;
    if (N == 64)
      fft_wave_one<INV, 1>(src, dst, N, tw, lane);
    else
      fft_wave_one<INV, 2>(src, dst, N, tw, lane);
  }
  __syncthreads();
  return b;
}

// Complex FFT of length N = 2^logN (r3 = 0) or N = 3 * 2^logN (r3 = 1):
// lengths 64 and 128 (blocks of 64 and 128 samples) by wavefronts with lane
// shuffles, the others by the LDS Stockham routines.  (Longer wave variants,
// 4 or 8 values per lane, raised the block kernel to 164 VGPRs for every
// workgroup, the bandwidth-bound tails included.)
template <bool INV>
__device__ __forceinline__ float2* fft_any(float2* a, float2* b, int N, int logN, int r3,
                                           const float2* __restrict__ tw, int nb = 1) {
  if (r3) return fft_stockham3<INV>(a, b, N, logN, tw, nb);
  if (N == 64 || N == 128) return fft_wave<INV>(a, b, N, tw, nb);
  return fft_stockham<INV>(a, b, N, logN, tw, nb);
}

// Packed spectra of nb real signals of 2P samples whose complex FFTs Z
// (length P each, [nb][P]) are in `Z`; writes [nb][P] packed bins to `X`
// (must not alias Z).  tw2 = W_2P^k table.  Ends with a barrier.
__device__ __forceinline__ void rfft_post(const float2* Z, float2* X, int P,
                                          const float2* __restrict__ tw2, int nb = 1) {
  const int per = (P >> 1) + 1;
  for (int w = threadIdx.x; w < nb * per; w += blockDim.x) {
    const int bb = w / per, k = w - bb * per;
    const float2* Zb = Z + bb * P;
    float2* Xb = X + bb * P;
    if (k == 0) {
      const float2 z = Zb[0];
      Xb[0] = make_float2(z.x + z.y, z.x - z.y);
      continue;
    }
    const float2 zk = Zb[k], zm = cconj(Zb[P - k]);
    const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    const float2 d = csub(zk, zm);
    const float2 O = make_float2(0.5f * d.y, -0.5f * d.x);  // -i d / 2
    const float2 wO = cmul(tw2[k], O);
    Xb[k] = cadd(E, wO);
    if (k != P - k) Xb[P - k] = cconj(csub(E, wO));
  }
  __syncthreads();
}

// Inverse of rfft_post without the 1/2 factors, for nb spectra [nb][P]:
// builds Z' = 2 Z so that IFFT_P(Z') / (2P) = z, z[m] = w[2m] + i w[2m+1].
// Ends with a barrier.
__device__ __forceinline__ void irfft_pre(const float2* X, float2* Z, int P,
                                          const float2* __restrict__ tw2, int nb = 1) {
  const int per = (P >> 1) + 1;
  for (int w = threadIdx.x; w < nb * per; w += blockDim.x) {
    const int bb = w / per, k = w - bb * per;
    const float2* Xb = X + bb * P;
    float2* Zb = Z + bb * P;
    if (k == 0) {
      const float2 x = Xb[0];  // (DC, Nyquist)
      Zb[0] = make_float2(x.x + x.y, x.x - x.y);
      continue;
    }
    const float2 xk = Xb[k], xm = cconj(Xb[P - k]);
    const float2 E = cadd(xk, xm);
    const float2 O = cmul(csub(xk, xm), cconj(tw2[k]));
    const float2 iO = make_float2(-O.y, O.x);
    Zb[k] = cadd(E, iO);
    if (k != P - k) {
      const float2 iOc = make_float2(O.y, O.x);  // i * conj(O)
      Zb[P - k] = cadd(cconj(E), iOc);
    }
  }
  __syncthreads();
}

}  // namespace rta
