// rta.hip -- host runtime and C ABI of librta (see include/rta.h).
//
// A context owns, on one device:
//   - the filter spectra of every tier, rows [pair][partition][P bins] in the
//     chosen storage type (built on the GPU at creation by k_spectra), plus a
//     dense copy of partitions 0 and 1 of every pair for the head
//     workgroups;
//   - per tier an FDL ring [Q][K][P] of FP32 input spectra and a partial-sum
//     area double-buffered by block parity; the input history ring
//     [Q][hist_len]; per later tier an output ring [L][ring_len];
//   - the tail work list, built once at creation and checked against every
//     buffer bound;
//   - pinned, device-mapped input/output/flag buffers for rta_process.
// Each block is one k_block launch on a stream; the block index is kept on
// the host and passed by value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rta.h"
#include "kernels.hpp"

using namespace rta;

namespace {

constexpr int kMinBlock = 16;
constexpr int kMaxBlock = 4096;
constexpr int kXcds = 8;                     // MI355X: 8 XCDs, workgroups round-robin
constexpr int64_t kStageBytes = 64ll << 20;  // filter taps staged per spectra batch
constexpr size_t kMaxTimedBlocks = 65536;

struct TierHost {
  int P = 0, logP = 0, K = 0, count = 0;
  int64_t offset = 0;
  void* H = nullptr;
  int64_t* pair_row = nullptr;
  int32_t* pair_K = nullptr;
  float2* X = nullptr;
  float2* partial = nullptr;
  float2* tw = nullptr;
  float* oring = nullptr;
  int nslots = 0;
  std::vector<int64_t> row;  // host copies
  std::vector<int32_t> kp;
};

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

struct rta_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  double fs = 0;
  int B = 0, Q = 0, L = 0, dtype = 0;
  uint32_t flags = 0;
  int n_tiers = 0;
  TierHost tier[kMaxTiers];
  int G = 1, rows_per_item = 0, n_phase = 1, max_items = 0, n_items = 0;
  int tail_items = 1024, tier_rows = 16;
  int n_groups = 0, head_slots = 0, head_nq = 1;
  int64_t hist_len = 0, ring_len = 0;
  size_t lds = 0;              // k_block dynamic LDS
  int64_t block = 0;           // index of the next block

  void* H01 = nullptr;         // [L][Q][2][P] partitions 0 and 1
  Item* tier_items = nullptr;  // k_tier lists [n_phase][max_tier_items]
  int32_t* tier_count = nullptr;
  int32_t* tier_slot0 = nullptr;
  int32_t* tier_nslot = nullptr;
  int max_tier_items = 0;
  std::vector<int32_t> tier_count_host;  // k_tier items per phase
  size_t lds_tier = 0;         // k_tier dynamic LDS
  float* hist = nullptr;
  Item* items = nullptr;
  int32_t* phase_count = nullptr;
  Group* groups = nullptr;
  unsigned int* head_count = nullptr;

  float* h_in = nullptr;       // pinned host staging, mapped into the device
  float* h_out = nullptr;
  int64_t* h_flag = nullptr;
  float* m_in = nullptr;       // device addresses of the three
  float* m_out = nullptr;
  int64_t* m_flag = nullptr;

  rta_ctx* fc = nullptr;        // feedback convolution: outputs -> inputs
  float* d_y = nullptr;         // [L][B] copy of the output block (its input)
  float* d_c = nullptr;         // [Q][B] its output, subtracted next block

  bool poisoned = false;
  bool timing = false;
  std::vector<hipEvent_t> events;  // 2 per timed block
  size_t events_used = 0;
  int64_t device_bytes = 0, spectra_bytes = 0;
  double h_bytes = 0, x_bytes = 0, io_bytes = 0, cmacs = 0, tail_bytes = 0;
  std::vector<void*> dev_allocs;
};

namespace {

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) {                                  \
      if (std::getenv("RTA_LOG"))                            \
        std::fprintf(stderr, "rta: %s failed: %s\n", #expr,  \
                     hipGetErrorString(e_));                 \
      (ctx)->poisoned = true;                                \
      return RTA_E_DEVICE;                                   \
    }                                                        \
  } while (0)

template <typename T>
int dev_alloc(rta_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return RTA_E_NOMEM;
  }
  c->dev_allocs.push_back(v);
  c->device_bytes += (int64_t)(count * sizeof(T));
  *p = static_cast<T*>(v);
  return RTA_OK;
}

size_t spectra_elem_bytes(int dtype) { return dtype == RTA_FP32 ? 8 : 4; }
int vec_bins(int dtype) { return dtype == RTA_FP32 ? 2 : 4; }

// W_P^j (j < P) then W_2P^k (k < P), FP64 evaluated then rounded to FP32.
std::vector<float2> twiddles(int P) {
  std::vector<float2> t(2 * (size_t)P);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < P; ++j) {
    const double a = -2.0 * pi * (double)j / (double)P;
    t[j] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  for (int k = 0; k < P; ++k) {
    const double a = -pi * (double)k / (double)P;
    t[P + k] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return t;
}

using BlockKernel = void (*)(const KArgs);

BlockKernel block_kernel(int dtype, int G) {
#define RTA_PICK(HT)                                   \
  switch (G) {                                         \
    case 1: return k_block<HT, 1>;                     \
    case 2: return k_block<HT, 2>;                     \
    case 4: return k_block<HT, 4>;                     \
    default: return nullptr;                           \
  }
  if (dtype == RTA_FP32) RTA_PICK(float2)
  if (dtype == RTA_FP16) RTA_PICK(f16c_t)
  if (dtype == RTA_BF16) RTA_PICK(bf16c_t)
#undef RTA_PICK
  return nullptr;
}

BlockKernel tier_kernel(int G) {
  switch (G) {
    case 1: return k_tier<1>;
    case 2: return k_tier<2>;
    case 4: return k_tier<4>;
    default: return nullptr;
  }
}

hipError_t launch_spectra(int dtype, dim3 grid, size_t lds, hipStream_t s, const float* taps,
                          const SpecRow* rows, void* H, int P, int logP, const float2* tw,
                          int* range) {
  if (dtype == RTA_FP32)
    hipLaunchKernelGGL(k_spectra<float2>, grid, dim3(kThreads), lds, s, taps, rows,
                       static_cast<float2*>(H), P, logP, tw, range);
  else if (dtype == RTA_FP16)
    hipLaunchKernelGGL(k_spectra<f16c_t>, grid, dim3(kThreads), lds, s, taps, rows,
                       static_cast<f16c_t*>(H), P, logP, tw, range);
  else
    hipLaunchKernelGGL(k_spectra<bf16c_t>, grid, dim3(kThreads), lds, s, taps, rows,
                       static_cast<bf16c_t*>(H), P, logP, tw, range);
  return hipGetLastError();
}

hipError_t launch_gather(int dtype, const TierHost& T, int n_pairs, void* H01, hipStream_t s) {
  const dim3 grid(2 * n_pairs);
  if (dtype == RTA_FP32)
    hipLaunchKernelGGL(k_gather_head_rows<float2>, grid, dim3(kThreads), 0, s,
                       static_cast<const float2*>(T.H), T.pair_row, T.pair_K, T.P, n_pairs,
                       static_cast<float2*>(H01));
  else if (dtype == RTA_FP16)
    hipLaunchKernelGGL(k_gather_head_rows<f16c_t>, grid, dim3(kThreads), 0, s,
                       static_cast<const f16c_t*>(T.H), T.pair_row, T.pair_K, T.P, n_pairs,
                       static_cast<f16c_t*>(H01));
  else
    hipLaunchKernelGGL(k_gather_head_rows<bf16c_t>, grid, dim3(kThreads), 0, s,
                       static_cast<const bf16c_t*>(T.H), T.pair_row, T.pair_K, T.P, n_pairs,
                       static_cast<bf16c_t*>(H01));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Argument validation (no HIP calls).
// ---------------------------------------------------------------------------
int validate(double fs, int32_t block, const rta_scheme* scheme, int32_t n_in, int32_t n_out,
             const float* const* filters, const int64_t* lengths, int32_t spectra,
             uint32_t flags, std::vector<int>& size, std::vector<int>& count) {
  if (!(fs > 0.0) || !std::isfinite(fs)) return RTA_E_ARG;
  if (!is_pow2(block) || block < kMinBlock || block > kMaxBlock) return RTA_E_ARG;
  if (n_in < 1 || n_out < 1 || (int64_t)n_in * n_out > (1 << 20)) return RTA_E_ARG;
  if (filters == nullptr || lengths == nullptr) return RTA_E_ARG;
  if (spectra != RTA_FP32 && spectra != RTA_FP16 && spectra != RTA_BF16) return RTA_E_ARG;
  if (flags & ~RTA_FLAG_SPIKE) return RTA_E_ARG;
  int64_t max_len = 0;
  for (int64_t i = 0; i < (int64_t)n_in * n_out; ++i) {
    if (lengths[i] < 0 || lengths[i] > (int64_t(1) << 31)) return RTA_E_ARG;
    if (lengths[i] > 0 && filters[i] == nullptr) return RTA_E_ARG;
    max_len = std::max(max_len, lengths[i]);
  }
  size.clear();
  count.clear();
  if (scheme == nullptr) {
    size.push_back(block);
    count.push_back(0);
  } else {
    if (scheme->n_tiers < 1 || scheme->n_tiers > kMaxTiers) return RTA_E_ARG;
    if (scheme->size == nullptr || scheme->count == nullptr) return RTA_E_ARG;
    for (int t = 0; t < scheme->n_tiers; ++t) {
      size.push_back(scheme->size[t]);
      count.push_back(scheme->count[t]);
    }
  }
  const int T = (int)size.size();
  if (size[0] != block) return RTA_E_ARG;
  int64_t off = 0;
  for (int t = 0; t < T; ++t) {
    if (!is_pow2(size[t]) || size[t] % block != 0 || size[t] > (1 << 13)) return RTA_E_ARG;
    if (t > 0 && size[t] <= size[t - 1]) return RTA_E_ARG;
    if (count[t] < 0 || (count[t] == 0 && t != T - 1)) return RTA_E_ARG;
    // a later tier's frame needs one block for its FFT and at least one for
    // its multiply-accumulate before its first output sample is due
    if (t > 0 && off < (int64_t)size[t] + block) return RTA_E_ARG;
    off += (int64_t)count[t] * size[t];
  }
  if (count[T - 1] > 0 && max_len > off) return RTA_E_ARG;
  return RTA_OK;
}

// ---------------------------------------------------------------------------
// Work lists.  The block index n selects phase n mod n_phase (n_phase =
// P_max / B).  k_block's list for a phase holds
//   - the first tier's tail items (every phase): partitions p >= 2 of every
//     (output group, input), cut into chunks of about R rows and bin slices;
//     each chunk owns one partial slot of its group (the heads do p = 0, 1);
//   - the multiply-accumulate items of later tiers whose frame is being
//     accumulated in that block.
// k_tier's list for a phase holds the later tiers' FFT items (in the block a
// frame's input completes) and their final items (in the block after the
// frame's last multiply-accumulate).  Tier t (P_t = r B, offset o_t) gives a
// frame s = (o_t + B - P_t) / B blocks between input completion and first
// output; its multiply-accumulate is spread over nmac = min(s, r + 1) - 1
// blocks (1 with RTA_FLAG_SPIKE).
// ---------------------------------------------------------------------------
struct Bucket {
  int tier, q, p0, k0;
  std::vector<Item> items;
  int64_t rows = 0;
};

struct Plan {
  std::vector<std::vector<Item>> block;  // per phase: k_block tail items
  std::vector<std::vector<Item>> tier;   // per phase: k_tier items
  std::vector<Group> groups;
  std::vector<int32_t> tier_slot0, tier_nslot;  // [tier][group]
};

// nmac of tier t >= 1 (see above)
int tier_nmac(const rta_ctx* c, int t) {
  const TierHost& T = c->tier[t];
  const int r = T.P / c->B;
  const int64_t s = (T.offset + c->B - T.P) / c->B;
  if (c->flags & RTA_FLAG_SPIKE) return 1;
  return (int)std::min<int64_t>(s, r + 1) - 1;
}

// XCD-aware placement: a bucket's items (same tier, input, partitions and
// bins; different outputs) all get list positions with the same residue
// mod 8, so they run on one XCD and fetch their delay-line rows into one L2.
std::vector<Item> place_on_xcds(std::vector<Bucket>& buckets) {
  std::vector<std::vector<Item>> xl(kXcds);
  std::vector<int64_t> load(kXcds, 0);
  std::stable_sort(buckets.begin(), buckets.end(),
                   [](const Bucket& a, const Bucket& b) { return a.rows > b.rows; });
  for (auto& b : buckets) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (auto& it : b.items) xl[x].push_back(it);
    load[x] += b.rows;
  }
  size_t longest = 0;
  for (auto& v : xl) longest = std::max(longest, v.size());
  std::vector<Item> flat(longest * kXcds, Item{});
  for (auto& it : flat) it.kind = K_NOP;
  for (int x = 0; x < kXcds; ++x)
    for (size_t i = 0; i < xl[x].size(); ++i) flat[i * kXcds + x] = xl[x][i];
  while (!flat.empty() && flat.back().kind == K_NOP) flat.pop_back();
  return flat;
}

void add_to_bucket(std::vector<Bucket>& buckets, const Item& it, int nl) {
  auto bit = std::find_if(buckets.begin(), buckets.end(), [&](const Bucket& b) {
    return b.tier == it.tier && b.q == it.q && b.p0 == it.p0 && b.k0 == it.k0;
  });
  if (bit == buckets.end()) {
    buckets.push_back(Bucket{it.tier, it.q, it.p0, it.k0, {}, 0});
    bit = buckets.end() - 1;
  }
  bit->items.push_back(it);
  bit->rows += (int64_t)(it.p1 - it.p0) * nl;
}

int build_plan(rta_ctx* c, Plan& plan) {
  const int G = c->G;
  const int C = vec_bins(c->dtype);
  const int ngroups = (c->L + G - 1) / G;
  const int n_phase = c->tier[c->n_tiers - 1].P / c->B;
  c->n_phase = n_phase;
  plan.block.assign(n_phase, {});
  plan.tier.assign(n_phase, {});
  plan.groups.clear();
  plan.tier_slot0.assign((size_t)kMaxTiers * ngroups, 0);
  plan.tier_nslot.assign((size_t)kMaxTiers * ngroups, 0);
  for (int g = 0; g < ngroups; ++g) {
    Group gr{};
    gr.l0 = g * G;
    gr.nl = std::min(G, c->L - gr.l0);
    plan.groups.push_back(gr);
  }
  auto group_rows = [&](const TierHost& T, const Group& gr, int q) {
    int kg = 0;
    for (int l = gr.l0; l < gr.l0 + gr.nl; ++l) kg = std::max(kg, T.kp[l * c->Q + q]);
    return kg;
  };

  // ---- first tier: partitions >= 2, every phase
  std::vector<Item> tier0;
  {
    TierHost& T = c->tier[0];
    const int P = T.P, W = std::min(P, kThreads * C), nslice = P / W;
    int64_t total_rows = 0;
    for (const Group& gr : plan.groups)
      for (int q = 0; q < c->Q; ++q) total_rows += std::max(0, group_rows(T, gr, q) - 2);
    int R = c->rows_per_item;
    if (R <= 0) {
      const int64_t target_items = std::max(1, c->tail_items);
      R = (int)std::max<int64_t>(8, (total_rows * nslice + target_items - 1) / target_items);
    }
    c->rows_per_item = R;
    int slot = 0;
    for (int g = 0; g < ngroups; ++g) {
      Group& gr = plan.groups[g];
      gr.slot0 = slot;
      gr.nslot = 0;
      for (int q = 0; q < c->Q; ++q) {
        const int kg = group_rows(T, gr, q);
        if (kg <= 2) continue;  // partitions 0 and 1 are done by the heads
        const int rows = kg - 2;
        const int nch = (rows + R - 1) / R;
        for (int ch = 0; ch < nch; ++ch) {
          const int p0 = 2 + (int)((int64_t)ch * rows / nch);
          const int p1 = 2 + (int)((int64_t)(ch + 1) * rows / nch);
          for (int sl = 0; sl < nslice; ++sl) {
            Item it{};
            it.kind = K_MAC;
            it.tier = 0;
            it.group = g;
            it.q = q;
            it.p0 = p0;
            it.p1 = p1;
            it.k0 = sl * W;
            it.slot = slot;
            tier0.push_back(it);
          }
          ++slot;
          ++gr.nslot;
        }
      }
    }
    T.nslots = slot;
  }

  // ---- later tiers
  std::vector<std::vector<Item>> tier_mac(n_phase);
  for (int t = 1; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    const int P = T.P, W = std::min(P, kThreads * C), nslice = P / W;
    const int r = P / c->B;
    const int nmac = tier_nmac(c, t);
    if (nmac < 1) return RTA_E_STATE;
    const int R = std::max(1, c->tier_rows);
    struct Chunk { int g, q, p0, p1, slot; };
    std::vector<Chunk> chunks;
    int slot = 0;
    for (int g = 0; g < ngroups; ++g) {
      const Group& gr = plan.groups[g];
      plan.tier_slot0[(size_t)t * ngroups + g] = slot;
      for (int q = 0; q < c->Q; ++q) {
        const int kg = group_rows(T, gr, q);
        if (kg == 0) continue;
        const int nch = (kg + R - 1) / R;
        for (int ch = 0; ch < nch; ++ch)
          chunks.push_back(Chunk{g, q, (int)((int64_t)ch * kg / nch),
                                 (int)((int64_t)(ch + 1) * kg / nch), slot++});
      }
      plan.tier_nslot[(size_t)t * ngroups + g] = slot - plan.tier_slot0[(size_t)t * ngroups + g];
    }
    T.nslots = slot;
    // spread the chunks over the nmac blocks, balancing rows
    int64_t total = 0;
    for (const Chunk& ch : chunks) total += ch.p1 - ch.p0;
    std::vector<int> when(chunks.size(), 0);
    int64_t acc = 0;
    for (size_t i = 0; i < chunks.size(); ++i) {
      when[i] = total > 0 ? (int)std::min<int64_t>(nmac - 1, acc * nmac / total) : 0;
      acc += chunks[i].p1 - chunks[i].p0;
    }
    for (int ph0 = r - 1; ph0 < n_phase; ph0 += r) {  // phases in which a frame completes
      for (int q = 0; q < c->Q; ++q) {
        bool used = false;
        for (int l = 0; l < c->L; ++l) used |= T.kp[l * c->Q + q] > 0;
        if (!used) continue;
        Item it{};
        it.kind = K_FFT;
        it.tier = t;
        it.q = q;
        it.lag = 0;
        plan.tier[ph0].push_back(it);
      }
      for (size_t i = 0; i < chunks.size(); ++i) {
        const int lag = 1 + when[i];
        for (int sl = 0; sl < nslice; ++sl) {
          Item it{};
          it.kind = K_MAC;
          it.tier = t;
          it.group = chunks[i].g;
          it.q = chunks[i].q;
          it.p0 = chunks[i].p0;
          it.p1 = chunks[i].p1;
          it.k0 = sl * W;
          it.slot = chunks[i].slot;
          it.lag = lag;
          tier_mac[(ph0 + lag) % n_phase].push_back(it);
        }
      }
      for (int g = 0; g < ngroups; ++g) {
        if (plan.tier_nslot[(size_t)t * ngroups + g] == 0) continue;
        Item it{};
        it.kind = K_FINAL;
        it.tier = t;
        it.group = g;
        it.lag = nmac;
        plan.tier[(ph0 + nmac) % n_phase].push_back(it);
      }
    }
  }
  c->n_groups = ngroups;

  // ---- per-phase k_block lists, XCD-aware
  for (int ph = 0; ph < n_phase; ++ph) {
    std::vector<Bucket> buckets;
    for (const Item& it : tier0) add_to_bucket(buckets, it, plan.groups[it.group].nl);
    for (const Item& it : tier_mac[ph]) add_to_bucket(buckets, it, plan.groups[it.group].nl);
    plan.block[ph] = place_on_xcds(buckets);
  }

  // every index the kernels derive from an item must stay inside the
  // buffers allocated for this plan
  for (const Group& gr : plan.groups)
    if (gr.l0 < 0 || gr.nl < 1 || gr.nl > G || gr.l0 + gr.nl > c->L || gr.slot0 < 0 ||
        gr.nslot < 0 || gr.slot0 + gr.nslot > c->tier[0].nslots)
      return RTA_E_STATE;
  for (int t = 1; t < c->n_tiers; ++t)
    for (int g = 0; g < ngroups; ++g) {
      const int s0 = plan.tier_slot0[(size_t)t * ngroups + g], ns = plan.tier_nslot[(size_t)t * ngroups + g];
      if (s0 < 0 || ns < 0 || s0 + ns > c->tier[t].nslots) return RTA_E_STATE;
    }
  for (int ph = 0; ph < n_phase; ++ph) {
    for (const Item& it : plan.block[ph]) {
      if (it.kind == K_NOP) continue;
      if (it.kind != K_MAC || it.tier < 0 || it.tier >= c->n_tiers) return RTA_E_STATE;
      if (it.group < 0 || it.group >= ngroups) return RTA_E_STATE;
      const TierHost& T = c->tier[it.tier];
      const int W = std::min(T.P, kThreads * C);
      if (it.q < 0 || it.q >= c->Q) return RTA_E_STATE;
      if (it.p0 < (it.tier == 0 ? 2 : 0) || it.p1 < it.p0 || it.p1 > T.K) return RTA_E_STATE;
      if (it.k0 < 0 || it.k0 % W != 0 || it.k0 + W > T.P) return RTA_E_STATE;
      if (it.tier == 0) {
        const Group& gr = plan.groups[it.group];
        if (it.slot < gr.slot0 || it.slot >= gr.slot0 + gr.nslot) return RTA_E_STATE;
      } else {
        const int s0 = plan.tier_slot0[(size_t)it.tier * ngroups + it.group];
        const int ns = plan.tier_nslot[(size_t)it.tier * ngroups + it.group];
        if (it.slot < s0 || it.slot >= s0 + ns) return RTA_E_STATE;
        if (it.lag < 1 || it.lag > T.P / c->B) return RTA_E_STATE;
      }
    }
    for (const Item& it : plan.tier[ph]) {
      if (it.tier < 1 || it.tier >= c->n_tiers) return RTA_E_STATE;
      if (it.kind == K_FFT && (it.q < 0 || it.q >= c->Q || it.lag != 0)) return RTA_E_STATE;
      if (it.kind == K_FINAL && (it.group < 0 || it.group >= ngroups || it.lag < 1)) return RTA_E_STATE;
      if (it.kind != K_FFT && it.kind != K_FINAL) return RTA_E_STATE;
    }
  }
  return RTA_OK;
}

KArgs make_args(const rta_ctx* c, const float* in, float* out, int64_t n) {
  KArgs a{};
  for (int t = 0; t < c->n_tiers; ++t) {
    const TierHost& T = c->tier[t];
    DevTier& d = a.tier[t];
    d.H = T.H;
    d.pair_row = T.pair_row;
    d.pair_K = T.pair_K;
    d.X = T.X;
    d.partial = T.partial;
    d.tw = T.tw;
    d.oring = T.oring;
    d.offset = T.offset;
    d.P = T.P;
    d.logP = T.logP;
    d.K = T.K;
    d.nslots = std::max(1, T.nslots);
    d.r = T.P / c->B;
  }
  a.items = c->items;
  a.phase_count = c->phase_count;
  a.groups = c->groups;
  a.hist = c->hist;
  a.in = in;
  a.out = out;
  a.hist_mask = c->hist_len - 1;
  a.ring_mask = c->ring_len - 1;
  a.B = c->B;
  a.Q = c->Q;
  a.L = c->L;
  a.n_tiers = c->n_tiers;
  a.n_phase = c->n_phase;
  a.max_items = c->max_items;
  a.head_nq = c->head_nq;
  a.n_head = c->n_groups;
  a.head_slots = c->head_slots;
  a.n = n;
  a.H01 = c->H01;
  a.head_count = c->head_count;
  a.done_flag = nullptr;  // set by rta_process, which polls it
  a.tier_items = c->tier_items;
  a.tier_count = c->tier_count;
  a.tier_slot0 = c->tier_slot0;
  a.tier_nslot = c->tier_nslot;
  a.max_tier_items = c->max_tier_items;
  a.n_groups_total = c->n_groups;
  return a;
}

// One block: heads of block n and tails of block n + 1 in a single launch,
// then, in blocks with later-tier FFTs or finals, one k_tier launch.
// `flag`: raise the host-visible completion flag (rta_process).
int launch_block(rta_ctx* c, const float* in, float* out, hipStream_t s, bool flag = false) {
  KArgs a = make_args(c, in, out, c->block);
  if (flag) a.done_flag = c->m_flag;
  const unsigned grid = (unsigned)(c->head_slots + c->max_items);
  const int phase = (int)(c->block % c->n_phase);
  const int n_tier = c->tier_count_host.empty() ? 0 : c->tier_count_host[phase];
  hipEvent_t* e = nullptr;
  if (c->timing && c->events_used + 2 <= 2 * kMaxTimedBlocks) {
    while (c->events.size() < c->events_used + 2) {
      hipEvent_t ev;
      HIP_TRY(c, hipEventCreate(&ev));
      c->events.push_back(ev);
    }
    e = &c->events[c->events_used];
    c->events_used += 2;
    HIP_TRY(c, hipEventRecord(e[0], s));
  }
  if (c->fc != nullptr) {
    a.sub = c->d_c;
    a.out2 = c->d_y;
  }
  hipLaunchKernelGGL(block_kernel(c->dtype, c->G), dim3(grid), dim3(kThreads), c->lds, s, a);
  HIP_TRY(c, hipGetLastError());
  if (n_tier > 0) {
    hipLaunchKernelGGL(tier_kernel(c->G), dim3(n_tier), dim3(kThreads), c->lds_tier, s, a);
    HIP_TRY(c, hipGetLastError());
  }
  if (c->fc != nullptr) {  // feedback estimate of this block, for the next one
    const int st = launch_block(c->fc, c->d_y, c->d_c, s);
    if (st != RTA_OK) {
      c->poisoned = true;
      return st;
    }
  }
  if (e) HIP_TRY(c, hipEventRecord(e[1], s));
  c->block += 1;
  return RTA_OK;
}

int zero_state(rta_ctx* c) {
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    HIP_TRY(c, hipMemsetAsync(T.X, 0, sizeof(float2) * (size_t)c->Q * T.K * T.P, c->stream));
    // before the first block the terms p >= 2 are all zero (zero history)
    HIP_TRY(c, hipMemsetAsync(T.partial, 0,
                              sizeof(float2) * (t == 0 ? 2 : 1) * (size_t)std::max(1, T.nslots) * c->G * T.P,
                              c->stream));
    if (T.oring)
      HIP_TRY(c, hipMemsetAsync(T.oring, 0, sizeof(float) * (size_t)c->L * c->ring_len, c->stream));
  }
  HIP_TRY(c, hipMemsetAsync(c->hist, 0, sizeof(float) * (size_t)c->Q * c->hist_len, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->head_count, 0, sizeof(unsigned int), c->stream));
  if (c->d_c) HIP_TRY(c, hipMemsetAsync(c->d_c, 0, sizeof(float) * (size_t)c->Q * c->B, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->fc) {
    const int st = zero_state(c->fc);
    if (st != RTA_OK) return st;
  }
  __atomic_store_n(c->h_flag, (int64_t)0, __ATOMIC_RELEASE);
  c->block = 0;
  return RTA_OK;
}

// Temporary device buffer released when it goes out of scope.
struct TmpDev {
  void* p = nullptr;
  ~TmpDev() {
    if (p) (void)hipFree(p);
  }
};

int build_spectra(rta_ctx* c, const float* const* filters, const int64_t* lengths) {
  int64_t max_len = 0;
  for (int64_t i = 0; i < (int64_t)c->Q * c->L; ++i) max_len = std::max(max_len, lengths[i]);
  const int64_t stage_floats = std::max<int64_t>(max_len, kStageBytes / 4);
  TmpDev stage, drows, drange;
  if (hipMalloc(&stage.p, sizeof(float) * (size_t)stage_floats) != hipSuccess ||
      hipMalloc(&drange.p, sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    return RTA_E_NOMEM;
  }
  HIP_TRY(c, hipMemsetAsync(drange.p, 0, sizeof(int), c->stream));

  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    const int P = T.P;
    const size_t lds = sizeof(float2) * 2 * (size_t)P;
    // a batch holds at most stage_floats taps, hence at most this many rows
    const int64_t row_cap = stage_floats / P + (int64_t)c->Q * c->L + 1;
    if (drows.p) { (void)hipFree(drows.p); drows.p = nullptr; }
    if (hipMalloc(&drows.p, sizeof(SpecRow) * (size_t)row_cap) != hipSuccess) {
      (void)hipGetLastError();
      return RTA_E_NOMEM;
    }
    std::vector<SpecRow> rows;
    std::vector<float> host_stage;
    auto flush = [&]() -> int {
      if (rows.empty()) return RTA_OK;
      HIP_TRY(c, hipMemcpyAsync(stage.p, host_stage.data(), sizeof(float) * host_stage.size(),
                                hipMemcpyHostToDevice, c->stream));
      HIP_TRY(c, hipMemcpyAsync(drows.p, rows.data(), sizeof(SpecRow) * rows.size(),
                                hipMemcpyHostToDevice, c->stream));
      HIP_TRY(c, launch_spectra(c->dtype, dim3((unsigned)rows.size()), lds, c->stream,
                                static_cast<const float*>(stage.p),
                                static_cast<const SpecRow*>(drows.p), T.H, P, T.logP, T.tw,
                                static_cast<int*>(drange.p)));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      rows.clear();
      host_stage.clear();
      return RTA_OK;
    };
    int st;
    for (int l = 0; l < c->L; ++l)
      for (int q = 0; q < c->Q; ++q) {
        const int pair_in = q * c->L + l;  // caller layout [in][out]
        const int pair = l * c->Q + q;     // device layout [out][in]
        const int kp = T.kp[pair];
        if (kp == 0) continue;
        const int64_t len = lengths[pair_in];
        const int64_t a0 = T.offset, a1 = std::min(len, T.offset + (int64_t)kp * P);
        const int64_t n = a1 - a0;
        if ((int64_t)host_stage.size() + n > stage_floats || (int64_t)rows.size() + kp > row_cap)
          if ((st = flush()) != RTA_OK) return st;
        const int64_t base = (int64_t)host_stage.size();
        host_stage.insert(host_stage.end(), filters[pair_in] + a0, filters[pair_in] + a1);
        for (int p = 0; p < kp; ++p) {
          SpecRow r{};
          r.src = base + (int64_t)p * P;
          r.len = (int32_t)std::max<int64_t>(0, std::min<int64_t>(P, n - (int64_t)p * P));
          r.dst = T.row[pair] + p;
          rows.push_back(r);
        }
      }
    if ((st = flush()) != RTA_OK) return st;
  }
  int range = 0;
  HIP_TRY(c, hipMemcpy(&range, drange.p, sizeof(int), hipMemcpyDeviceToHost));
  return range ? RTA_E_RANGE : RTA_OK;
}

int create_impl(rta_ctx* c, const std::vector<int>& size, const std::vector<int>& count,
                const float* const* filters, const int64_t* lengths) {
  int st;
  HIP_TRY(c, hipGetDevice(&c->device));
  HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));

  // tiers and partition counts
  c->n_tiers = (int)size.size();
  int64_t off = 0;
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    T.P = size[t];
    T.logP = ilog2(T.P);
    T.offset = off;
    T.row.assign((size_t)c->Q * c->L, -1);
    T.kp.assign((size_t)c->Q * c->L, 0);
    int64_t rows = 0;
    int kmax = 0;
    for (int l = 0; l < c->L; ++l)
      for (int q = 0; q < c->Q; ++q) {
        const int64_t len = lengths[q * c->L + l];
        int64_t need = len > off ? (len - off + T.P - 1) / T.P : 0;
        if (count[t] > 0) need = std::min<int64_t>(need, count[t]);
        const int pair = l * c->Q + q;
        T.kp[pair] = (int)need;
        if (need > 0) {
          T.row[pair] = rows;
          rows += need;
        }
        kmax = std::max<int>(kmax, (int)need);
      }
    T.count = count[t] > 0 ? count[t] : kmax;
    T.K = std::max(1, kmax);
    off += (int64_t)T.count * T.P;
    const size_t eb = spectra_elem_bytes(c->dtype);
    const double per_block = (double)c->B / T.P;  // a tier's frame recurs every P/B blocks
    c->spectra_bytes += rows * T.P * (int64_t)eb;
    c->h_bytes += (double)rows * T.P * eb * per_block;
    c->cmacs += (double)rows * T.P * per_block;
    c->x_bytes += (double)c->Q * kmax * T.P * 8.0 * per_block;
    if (t == 0) {
      double tail_rows = 0;
      for (int32_t kp : T.kp) tail_rows += std::max(0, kp - 2);
      c->tail_bytes = tail_rows * T.P * eb + (double)c->Q * std::max(0, kmax - 2) * T.P * 8.0;
    }
    if ((st = dev_alloc(c, reinterpret_cast<char**>(&T.H), (size_t)std::max<int64_t>(1, rows) * T.P * eb)) != RTA_OK)
      return st;
    if ((st = dev_alloc(c, &T.pair_row, T.row.size())) != RTA_OK) return st;
    if ((st = dev_alloc(c, &T.pair_K, T.kp.size())) != RTA_OK) return st;
    if ((st = dev_alloc(c, &T.X, (size_t)c->Q * T.K * T.P)) != RTA_OK) return st;
    if ((st = dev_alloc(c, &T.tw, 2 * (size_t)T.P)) != RTA_OK) return st;
    HIP_TRY(c, hipMemcpy(T.pair_row, T.row.data(), sizeof(int64_t) * T.row.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(T.pair_K, T.kp.data(), sizeof(int32_t) * T.kp.size(), hipMemcpyHostToDevice));
    const std::vector<float2> tw = twiddles(T.P);
    HIP_TRY(c, hipMemcpy(T.tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice));
  }
  c->io_bytes = 4.0 * c->B * (c->Q + c->L);
  c->hist_len = std::max<int64_t>(2 * c->B, 2 * (int64_t)c->tier[c->n_tiers - 1].P);
  c->hist_len = int64_t(1) << ilog2(c->hist_len);
  // later tiers store each frame's output up to o_t samples ahead of the
  // block being emitted (their time-domain delay)
  c->ring_len = 1;
  if (c->n_tiers > 1) c->ring_len = int64_t(1) << ilog2(c->tier[c->n_tiers - 1].offset + 2 * c->B);
  for (int t = 1; t < c->n_tiers; ++t)
    if ((st = dev_alloc(c, &c->tier[t].oring, (size_t)c->L * c->ring_len)) != RTA_OK) return st;

  // spectra, then the heads' dense copy of partitions 0 and 1
  if ((st = build_spectra(c, filters, lengths)) != RTA_OK) return st;
  const size_t eb = spectra_elem_bytes(c->dtype);
  if ((st = dev_alloc(c, reinterpret_cast<char**>(&c->H01), (size_t)c->L * c->Q * 2 * c->tier[0].P * eb)) != RTA_OK)
    return st;
  HIP_TRY(c, launch_gather(c->dtype, c->tier[0], c->L * c->Q, c->H01, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  // outputs per group: as requested, halved until a head's LDS fits
  int max_lds = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  while (c->G > 1 && (int64_t)sizeof(float2) * head_lds(c->tier[0].P, c->G, 1).total + 64 > max_lds)
    c->G /= 2;

  // work lists
  Plan plan;
  if ((st = build_plan(c, plan)) != RTA_OK) return st;
  c->n_groups = (int)plan.groups.size();
  c->head_slots = (c->n_groups + kXcds - 1) / kXcds * kXcds;  // keeps tails' XCD residues
  size_t mb = 1, mt = 1;
  for (int ph = 0; ph < c->n_phase; ++ph) {
    mb = std::max(mb, plan.block[ph].size());
    mt = std::max(mt, plan.tier[ph].size());
  }
  c->max_items = (int)mb;
  c->max_tier_items = (int)mt;
  c->n_items = (int)plan.block[0].size();
  std::vector<Item> all_b((size_t)c->n_phase * mb, Item{}), all_t((size_t)c->n_phase * mt, Item{});
  std::vector<int32_t> cnt_b(c->n_phase), cnt_t(c->n_phase);
  for (auto& it : all_b) it.kind = K_NOP;
  for (auto& it : all_t) it.kind = K_NOP;
  for (int ph = 0; ph < c->n_phase; ++ph) {
    std::copy(plan.block[ph].begin(), plan.block[ph].end(), all_b.begin() + (size_t)ph * mb);
    std::copy(plan.tier[ph].begin(), plan.tier[ph].end(), all_t.begin() + (size_t)ph * mt);
    cnt_b[ph] = (int32_t)plan.block[ph].size();
    cnt_t[ph] = (int32_t)plan.tier[ph].size();
  }
  c->tier_count_host = cnt_t;
  if ((st = dev_alloc(c, &c->items, all_b.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->phase_count, cnt_b.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_items, all_t.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_count, cnt_t.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_slot0, plan.tier_slot0.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_nslot, plan.tier_nslot.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->groups, plan.groups.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->head_count, 1)) != RTA_OK) return st;
  HIP_TRY(c, hipMemcpy(c->items, all_b.data(), sizeof(Item) * all_b.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->phase_count, cnt_b.data(), sizeof(int32_t) * cnt_b.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->tier_items, all_t.data(), sizeof(Item) * all_t.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->tier_count, cnt_t.data(), sizeof(int32_t) * cnt_t.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->tier_slot0, plan.tier_slot0.data(), sizeof(int32_t) * plan.tier_slot0.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->tier_nslot, plan.tier_nslot.data(), sizeof(int32_t) * plan.tier_nslot.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->groups, plan.groups.data(), sizeof(Group) * plan.groups.size(), hipMemcpyHostToDevice));

  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    const size_t bufs = t == 0 ? 2 : 1;  // the first tier's partials alternate by block parity
    if ((st = dev_alloc(c, &T.partial, bufs * (size_t)std::max(1, T.nslots) * c->G * T.P)) != RTA_OK)
      return st;
  }
  if ((st = dev_alloc(c, &c->hist, (size_t)c->Q * c->hist_len)) != RTA_OK) return st;

  // rta_process I/O and completion flag: pinned host memory that the kernel
  // reads and writes directly over PCIe (no DMA copies on the latency path)
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_in), sizeof(float) * (size_t)c->Q * c->B,
                    hipHostMallocMapped) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_out), sizeof(float) * (size_t)c->L * c->B,
                    hipHostMallocMapped) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_flag), sizeof(int64_t),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return RTA_E_NOMEM;
  }
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_in), c->h_in, 0));
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_out), c->h_out, 0));
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_flag), c->h_flag, 0));

  // LDS: the larger of a head's layout (HeadLds) and a tail item's row-group
  // reduction.  head_nq: as many inputs per pass as fit in 48 KB, at least 1.
  const int C = vec_bins(c->dtype);
  const int P0 = c->tier[0].P;
  const int fixed = head_lds(P0, c->G, 1).total - 2 * std::max(1, c->G) * P0;
  c->head_nq = std::max(1, std::min(c->Q, (6144 - fixed) / (2 * P0)));
  c->lds = sizeof(float2) * std::max((size_t)head_lds(P0, c->G, c->head_nq).total,
                                     (size_t)kThreads * C * c->G);
  if ((int64_t)c->lds + 64 > (int64_t)max_lds) return RTA_E_UNSUPPORTED;
  if (c->lds > 65536)
    HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(block_kernel(c->dtype, c->G)),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds));
  if (c->n_tiers > 1) {
    int pmax = 0;
    for (int t = 1; t < c->n_tiers; ++t) pmax = std::max(pmax, c->tier[t].P);
    c->lds_tier = sizeof(float2) * (size_t)tier_lds(pmax);
    if ((int64_t)c->lds_tier + 64 > (int64_t)max_lds) return RTA_E_UNSUPPORTED;
    if (c->lds_tier > 65536)
      HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(tier_kernel(c->G)),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_tier));
  }
  return zero_state(c);
}

void free_all(rta_ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->fc) {
    free_all(c->fc);
    delete c->fc;
    c->fc = nullptr;
  }
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  for (void* p : c->dev_allocs) (void)hipFree(p);
  c->dev_allocs.clear();
  if (c->h_in) (void)hipHostFree(c->h_in);
  if (c->h_out) (void)hipHostFree(c->h_out);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->stream) (void)hipStreamDestroy(c->stream);
}

}  // namespace

namespace {

// Candidate schemes of the autotuner: uniform, and for partition ratios 8
// and 4 the tiers B, rB, r^2 B, ... (<= 8192) with tier t >= 1 starting at
// 2 P_t - B, kept while the longest filter reaches them.
std::vector<std::vector<std::pair<int, int>>> scheme_candidates(int B, int64_t max_len) {
  std::vector<std::vector<std::pair<int, int>>> out;
  out.push_back({{B, 0}});
  for (int ratio : {8, 4}) {
    std::vector<std::pair<int, int>> sch;
    int64_t o = 0;
    int64_t P = B;
    while (true) {
      const int64_t Pn = P * ratio;
      const int64_t on = 2 * Pn - B;  // start of the next tier
      if (Pn > 8192 || max_len <= on) break;
      sch.push_back({(int)P, (int)((on - o) / P)});
      o = on;
      P = Pn;
    }
    if (sch.empty()) continue;
    sch.push_back({(int)P, 0});
    if (std::find(out.begin(), out.end(), sch) == out.end()) out.push_back(sch);
  }
  return out;
}

// Mean block time (us) of one context over `blocks` device-path blocks.
int time_blocks(rta_ctx* c, int blocks, double* us) {
  float* din = nullptr;
  float* dout = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = RTA_OK;
  float ms = 0.f;
  if (hipMalloc(&din, sizeof(float) * (size_t)c->Q * c->B) != hipSuccess ||
      hipMalloc(&dout, sizeof(float) * (size_t)c->L * c->B) != hipSuccess ||
      hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMemset(din, 0, sizeof(float) * (size_t)c->Q * c->B) != hipSuccess) {
    st = RTA_E_DEVICE;
  }
  for (int i = 0; st == RTA_OK && i < 16; ++i) st = rta_process_device(c, din, dout, s);
  if (st == RTA_OK && hipEventRecord(e0, s) != hipSuccess) st = RTA_E_DEVICE;
  for (int i = 0; st == RTA_OK && i < blocks; ++i) st = rta_process_device(c, din, dout, s);
  if (st == RTA_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    st = RTA_E_DEVICE;
  if (st == RTA_OK) *us = 1e3 * ms / blocks;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (din) (void)hipFree(din);
  if (dout) (void)hipFree(dout);
  (void)hipGetLastError();
  return st;
}

}  // namespace

extern "C" {

int rta_create_tuned(rta_ctx** out, double fs, int32_t block, const rta_scheme* scheme,
                     int32_t n_in, int32_t n_out, const float* const* filters,
                     const int64_t* lengths, int32_t spectra, uint32_t flags,
                     const rta_tuning* tuning) {
  if (out == nullptr) return RTA_E_ARG;
  *out = nullptr;
  std::vector<int> size, count;
  int st = validate(fs, block, scheme, n_in, n_out, filters, lengths, spectra, flags, size, count);
  if (st != RTA_OK) return st;
  if (tuning != nullptr) {
    const int g = tuning->outputs_per_group;
    if ((g != 0 && g != 1 && g != 2 && g != 4) || tuning->tail_items < 0 || tuning->tail_rows < 0 ||
        tuning->tier_rows < 0)
      return RTA_E_ARG;
  }
  rta_ctx* c = new (std::nothrow) rta_ctx();
  if (c == nullptr) return RTA_E_NOMEM;
  c->fs = fs;
  c->B = block;
  c->Q = n_in;
  c->L = n_out;
  c->dtype = spectra;
  c->flags = flags;
  // tiling defaults measured on the 1 -> 32 x 480,000-tap workload: two
  // outputs per workgroup and about 1,024 first-tier items
  c->G = n_out >= 16 ? 2 : 1;
  if (tuning != nullptr) {
    if (tuning->outputs_per_group) c->G = tuning->outputs_per_group;
    if (tuning->tail_items) c->tail_items = tuning->tail_items;
    if (tuning->tail_rows) c->rows_per_item = tuning->tail_rows;
    if (tuning->tier_rows) c->tier_rows = tuning->tier_rows;
  }
  st = create_impl(c, size, count, filters, lengths);
  if (st != RTA_OK) {
    free_all(c);
    delete c;
    return st;
  }
  *out = c;
  return RTA_OK;
}

int rta_create(rta_ctx** out, double fs, int32_t block, const rta_scheme* scheme, int32_t n_in,
               int32_t n_out, const float* const* filters, const int64_t* lengths,
               int32_t spectra, uint32_t flags) {
  return rta_create_tuned(out, fs, block, scheme, n_in, n_out, filters, lengths, spectra, flags,
                          nullptr);
}

int rta_process(rta_ctx* c, const float* in, float* out) {
  if (c == nullptr || in == nullptr || out == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  std::memcpy(c->h_in, in, sizeof(float) * (size_t)c->Q * c->B);
  const int64_t want = c->block + 1;
  int st = launch_block(c, c->m_in, c->m_out, c->stream, true);
  if (st != RTA_OK) return st;
  // spin until the last head has raised the flag; the tail workgroups of the
  // same launch keep running.  Every few thousand polls the stream is asked
  // for errors so a failed launch cannot spin forever.
  for (uint64_t i = 1;; ++i) {
    if (__atomic_load_n(c->h_flag, __ATOMIC_ACQUIRE) == want) break;
    if ((i & 4095) == 0) {
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipSuccess) {
        if (__atomic_load_n(c->h_flag, __ATOMIC_ACQUIRE) == want) break;
        c->poisoned = true;
        return RTA_E_DEVICE;
      }
      if (e != hipErrorNotReady) HIP_TRY(c, e);
    }
  }
  std::memcpy(out, c->h_out, sizeof(float) * (size_t)c->L * c->B);
  return RTA_OK;
}

int rta_process_device(rta_ctx* c, const float* d_in, float* d_out, void* stream) {
  if (c == nullptr || d_in == nullptr || d_out == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  return launch_block(c, d_in, d_out, static_cast<hipStream_t>(stream));
}

int rta_reset(rta_ctx* c) {
  if (c == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  HIP_TRY(c, hipDeviceSynchronize());
  return zero_state(c);
}

int rta_query(rta_ctx* c, rta_info* info) {
  if (c == nullptr || info == nullptr) return RTA_E_ARG;
  std::memset(info, 0, sizeof(*info));
  info->fs = c->fs;
  info->deadline_us = 1e6 * c->B / c->fs;
  info->block = c->B;
  info->n_in = c->Q;
  info->n_out = c->L;
  info->n_tiers = c->n_tiers;
  info->spectra_dtype = c->dtype;
  info->n_phases = c->n_phase;
  for (int t = 0; t < c->n_tiers; ++t) {
    info->tier_size[t] = c->tier[t].P;
    info->tier_count[t] = c->tier[t].count;
    info->tier_offset[t] = c->tier[t].offset;
  }
  info->blocks_done = c->block;
  info->spectra_bytes = c->spectra_bytes;
  info->device_bytes = c->device_bytes;
  info->h_bytes_per_block = c->h_bytes;
  info->x_bytes_per_block = c->x_bytes;
  info->io_bytes_per_block = c->io_bytes;
  info->cmacs_per_block = c->cmacs;
  info->tail_bytes_per_block = c->tail_bytes;
  info->grid = c->head_slots + c->max_items;
  info->outputs_per_group = c->G;
  info->rows_per_item = c->rows_per_item;
  info->poisoned = c->poisoned ? 1 : 0;
  return c->poisoned ? RTA_E_DEVICE : RTA_OK;
}

int rta_set_feedback(rta_ctx* c, const float* const* fb, const int64_t* lengths, int32_t spectra) {
  if (c == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  HIP_TRY(c, hipDeviceSynchronize());
  if (c->fc) {
    free_all(c->fc);
    delete c->fc;
    c->fc = nullptr;
  }
  if (fb != nullptr) {
    if (lengths == nullptr) return RTA_E_ARG;
    // the feedback convolution runs outputs -> inputs: its filter [l][q]
    // is f_ql
    const int64_t np = (int64_t)c->Q * c->L;
    std::vector<const float*> ft(np);
    std::vector<int64_t> lt(np);
    for (int q = 0; q < c->Q; ++q)
      for (int l = 0; l < c->L; ++l) {
        ft[(int64_t)l * c->Q + q] = fb[(int64_t)q * c->L + l];
        lt[(int64_t)l * c->Q + q] = lengths[(int64_t)q * c->L + l];
      }
    rta_ctx* fc = nullptr;
    const int st = rta_create_tuned(&fc, c->fs, c->B, nullptr, c->L, c->Q, ft.data(), lt.data(),
                                    spectra, 0, nullptr);
    if (st != RTA_OK) return st;
    c->fc = fc;
    if (c->d_y == nullptr) {
      int s2;
      if ((s2 = dev_alloc(c, &c->d_y, (size_t)c->L * c->B)) != RTA_OK) return s2;
      if ((s2 = dev_alloc(c, &c->d_c, (size_t)c->Q * c->B)) != RTA_OK) return s2;
    }
  }
  return zero_state(c);
}

int rta_timing_enable(rta_ctx* c, int32_t on) {
  if (c == nullptr) return RTA_E_ARG;
  c->timing = on != 0;
  return RTA_OK;
}

int rta_timing_read(rta_ctx* c, int64_t* blocks, double* block_ms) {
  if (c == nullptr || blocks == nullptr || block_ms == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  *blocks = 0;
  *block_ms = 0.0;
  for (size_t i = 0; i + 2 <= c->events_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(c, hipEventSynchronize(c->events[i + 1]));
    HIP_TRY(c, hipEventElapsedTime(&ms, c->events[i], c->events[i + 1]));
    *block_ms += ms;
    *blocks += 1;
  }
  c->events_used = 0;
  return RTA_OK;
}

int rta_probe_read(const void* d_buf, int64_t bytes, int32_t grid, float* d_sink, void* stream) {
  if (d_buf == nullptr || d_sink == nullptr || bytes < 16 || grid < 1) return RTA_E_ARG;
  if ((reinterpret_cast<uintptr_t>(d_buf) & 15) != 0) return RTA_E_ARG;
  hipLaunchKernelGGL(k_read_probe, dim3(grid), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                     static_cast<const f32x4*>(d_buf), bytes / 16, d_sink);
  return hipGetLastError() == hipSuccess ? RTA_OK : RTA_E_DEVICE;
}

int rta_autotune(double fs, int32_t block, const rta_scheme* scheme, int32_t n_in, int32_t n_out,
                 const float* const* filters, const int64_t* lengths, int32_t spectra,
                 uint32_t flags, int32_t blocks, rta_tuning* best, double* best_us) {
  if (best == nullptr || best_us == nullptr || blocks < 1) return RTA_E_ARG;
  std::vector<int> size, count;
  int st = validate(fs, block, scheme, n_in, n_out, filters, lengths, spectra, flags, size, count);
  if (st != RTA_OK) return st;
  int64_t max_len = 0;
  for (int64_t i = 0; i < (int64_t)n_in * n_out; ++i) max_len = std::max(max_len, lengths[i]);
  std::vector<std::vector<std::pair<int, int>>> schemes;
  if (scheme != nullptr) {
    std::vector<std::pair<int, int>> sch;
    for (size_t t = 0; t < size.size(); ++t) sch.push_back({size[t], count[t]});
    schemes.push_back(sch);
  } else {
    schemes = scheme_candidates(block, max_len);
  }
  auto trial = [&](const std::vector<std::pair<int, int>>& sch, const rta_tuning& tu, double* us) {
    std::vector<int32_t> sz, ct;
    for (auto& p : sch) {
      sz.push_back(p.first);
      ct.push_back(p.second);
    }
    rta_scheme rs{(int32_t)sch.size(), sz.data(), ct.data()};
    rta_ctx* c = nullptr;
    int s2 = rta_create_tuned(&c, fs, block, &rs, n_in, n_out, filters, lengths, spectra, flags, &tu);
    if (s2 != RTA_OK) return s2;
    s2 = time_blocks(c, blocks, us);
    rta_destroy(c);
    return s2;
  };
  // stage 1: the scheme, with default tiles; stage 2: the tiles, for that scheme
  double best_t = 1e300;
  size_t best_s = 0;
  for (size_t i = 0; i < schemes.size(); ++i) {
    double us = 0;
    const rta_tuning tu{};
    const int s2 = trial(schemes[i], tu, &us);
    if (s2 == RTA_E_DEVICE) return s2;
    if (s2 == RTA_OK && us < best_t) {
      best_t = us;
      best_s = i;
    }
  }
  if (best_t == 1e300) return RTA_E_UNSUPPORTED;
  rta_tuning bt{};
  for (int g : {1, 2, 4}) {
    if (g > n_out) continue;
    for (int items : {512, 1024, 2048}) {
      rta_tuning tu{};
      tu.outputs_per_group = g;
      tu.tail_items = items;
      double us = 0;
      const int s2 = trial(schemes[best_s], tu, &us);
      if (s2 == RTA_E_DEVICE) return s2;
      if (s2 == RTA_OK && us < best_t) {
        best_t = us;
        bt = tu;
      }
    }
  }
  bt.n_tiers = (int32_t)schemes[best_s].size();
  for (int t = 0; t < bt.n_tiers; ++t) {
    bt.size[t] = schemes[best_s][t].first;
    bt.count[t] = schemes[best_s][t].second;
  }
  *best = bt;
  *best_us = best_t;
  return RTA_OK;
}

int rta_destroy(rta_ctx* c) {
  if (c == nullptr) return RTA_OK;
  free_all(c);
  delete c;
  return RTA_OK;
}

const char* rta_strerror(int status) {
  switch (status) {
    case RTA_OK: return "ok";
    case RTA_E_ARG: return "invalid argument";
    case RTA_E_NOMEM: return "out of device or pinned host memory";
    case RTA_E_RANGE: return "filter spectrum exceeds the FP16 range";
    case RTA_E_DEVICE: return "HIP runtime error (context poisoned)";
    case RTA_E_STATE: return "call not valid in the current state";
    case RTA_E_UNSUPPORTED: return "not supported by this build";
    default: return "unknown status";
  }
}

}  // extern "C"
