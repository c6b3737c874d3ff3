// rta.hip -- host runtime and C ABI of librta (see include/rta.h).
//
// A context owns, on one device:
//   - the filter spectra of every tier, rows [pair][partition][P bins] in the
//     chosen storage type (built on the GPU at creation, k_spectra);
//   - per tier an FDL ring [Q][K][P] of FP32 input spectra and a partial-sum
//     area; the input history ring [Q][hist_len]; per later tier an output
//     ring [L][ring_len];
//   - the work lists: per block phase a list of items, one per workgroup of
//     the block launch, built here once and never changed;
//   - the device block index and arrival counters.
// rta_process() replays a captured graph (H2D input, block kernel, D2H
// output); rta_process_device() launches the block kernel on a caller stream.
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

int env_int(const char* name, int dflt) {
  const char* s = std::getenv(name);
  if (s == nullptr || *s == 0) return dflt;
  return std::atoi(s);
}

}  // namespace

struct rta_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  double fs = 0;
  int B = 0, Q = 0, L = 0, dtype = 0;
  uint32_t flags = 0;
  int n_tiers = 0;
  TierHost tier[kMaxTiers];
  int G = 1, rows_per_item = 0, grid = 0, n_phase = 1, max_items = 0;
  int64_t hist_len = 0, ring_len = 0;
  size_t lds_bytes = 0;        // k_mac dynamic LDS
  size_t lds_final_bytes = 0;  // k_final dynamic LDS

  float* hist = nullptr;
  Item* items = nullptr;
  int32_t* phase_count = nullptr;
  Group* groups = nullptr;
  DevState* state = nullptr;
  int n_groups = 0;

  float* d_in = nullptr;
  float* d_out = nullptr;
  float* h_in = nullptr;
  float* h_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  bool poisoned = false;
  bool timing = false;
  std::vector<hipEvent_t> events;  // 3 per timed block
  size_t events_used = 0;
  int64_t device_bytes = 0, spectra_bytes = 0;
  double h_bytes = 0, x_bytes = 0, io_bytes = 0, cmacs = 0;
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

BlockKernel mac_kernel(int dtype, int G) {
#define RTA_PICK(HT)                                   \
  switch (G) {                                         \
    case 1: return k_mac<HT, 1>;                       \
    case 2: return k_mac<HT, 2>;                       \
    case 4: return k_mac<HT, 4>;                       \
    default: return nullptr;                           \
  }
  if (dtype == RTA_FP32) RTA_PICK(float2)
  if (dtype == RTA_FP16) RTA_PICK(f16c_t)
  if (dtype == RTA_BF16) RTA_PICK(bf16c_t)
#undef RTA_PICK
  return nullptr;
}

BlockKernel final_kernel(int G) {
  switch (G) {
    case 1: return k_final<1>;
    case 2: return k_final<2>;
    case 4: return k_final<4>;
    default: return nullptr;
  }
}

int vec_bins(int dtype) { return dtype == RTA_FP32 ? 2 : 4; }

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
  if (flags & ~(RTA_FLAG_SPIKE | RTA_FLAG_NO_GRAPH)) return RTA_E_ARG;
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
    if (t > 0 && off < 2 * (int64_t)size[t] - block) return RTA_E_ARG;
    off += (int64_t)count[t] * size[t];
  }
  if (count[T - 1] > 0 && max_len > off) return RTA_E_ARG;
  if (T > 1) return RTA_E_UNSUPPORTED;  // later tiers: not built yet
  return RTA_OK;
}

// ---------------------------------------------------------------------------
// Work lists for the uniform first tier.
// ---------------------------------------------------------------------------
struct Bucket {
  int q, p0, k0;
  std::vector<Item> items;
  int64_t rows = 0;
};

int build_plan(rta_ctx* c, std::vector<Item>& flat, std::vector<Group>& groups) {
  TierHost& T = c->tier[0];
  const int P = T.P;
  const int C = vec_bins(c->dtype);
  const int W = std::min(P, kThreads * C);
  const int nslice = P / W;
  const int G = c->G;
  const int ngroups = (c->L + G - 1) / G;

  // total partition rows of the groups, to size the items
  int64_t total_rows = 0;
  for (int g = 0; g < ngroups; ++g)
    for (int q = 0; q < c->Q; ++q) {
      int kg = 0;
      for (int l = g * G; l < std::min(c->L, g * G + G); ++l) kg = std::max(kg, T.kp[l * c->Q + q]);
      total_rows += kg;
    }
  int R = c->rows_per_item;
  if (R <= 0) {
    const int64_t target_items = env_int("RTA_TARGET_ITEMS", 2048);
    R = (int)std::max<int64_t>(8, (total_rows * nslice + target_items - 1) / target_items);
  }
  c->rows_per_item = R;

  std::vector<Bucket> buckets;
  std::vector<int> writer_done(c->Q, 0);
  groups.clear();
  int slot = 0;
  for (int g = 0; g < ngroups; ++g) {
    Group gr;
    gr.l0 = g * G;
    gr.nl = std::min(G, c->L - gr.l0);
    gr.slot0 = slot;
    gr.nslot = 0;
    std::vector<std::pair<int, Item>> mine;  // bucket key index, item
    for (int q = 0; q < c->Q; ++q) {
      int kg = 0;
      for (int l = gr.l0; l < gr.l0 + gr.nl; ++l) kg = std::max(kg, T.kp[l * c->Q + q]);
      if (kg == 0) continue;
      const int nch = (kg + R - 1) / R;
      for (int ch = 0; ch < nch; ++ch) {
        const int p0 = (int)((int64_t)ch * kg / nch), p1 = (int)((int64_t)(ch + 1) * kg / nch);
        for (int sl = 0; sl < nslice; ++sl) {
          Item it{};
          it.kind = K_MAC0;
          it.tier = 0;
          it.group = g;
          it.q = q;
          it.p0 = p0;
          it.p1 = p1;
          it.k0 = sl * W;
          it.slot = slot;
          if (p0 == 0 && !writer_done[q]) {
            it.flags |= F_WRITE_X;
            if (sl == 0) it.flags |= F_WRITE_HIST;
          }
          mine.push_back({0, it});
        }
        ++slot;
        ++gr.nslot;
      }
      writer_done[q] = 1;
    }
    if (gr.nslot == 0) {  // an output with no path still emits every block
      Item it{};
      it.kind = K_MAC0;
      it.group = g;
      it.q = 0;
      it.p0 = it.p1 = 0;
      it.k0 = 0;
      it.slot = slot++;
      gr.nslot = 1;
      mine.push_back({0, it});
    }
    for (auto& m : mine) m.second.target = (int)mine.size();
    // bucket by (q, p0, k0): items that read the same delay-line rows
    for (auto& m : mine) {
      const Item& it = m.second;
      auto bit = std::find_if(buckets.begin(), buckets.end(), [&](const Bucket& b) {
        return b.q == it.q && b.p0 == it.p0 && b.k0 == it.k0;
      });
      if (bit == buckets.end()) {
        buckets.push_back(Bucket{it.q, it.p0, it.k0, {}, 0});
        bit = buckets.end() - 1;
      }
      bit->items.push_back(it);
      bit->rows += (int64_t)(it.p1 - it.p0) * gr.nl;
    }
    groups.push_back(gr);
  }
  T.nslots = slot;
  c->n_groups = (int)groups.size();

  // XCD-aware placement: a bucket's items all get list positions with the
  // same residue mod 8, so its delay-line rows are fetched into one L2.
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
  flat.assign(longest * kXcds, Item{});
  for (auto& it : flat) it.kind = K_NOP;
  for (int x = 0; x < kXcds; ++x)
    for (size_t i = 0; i < xl[x].size(); ++i) flat[i * kXcds + x] = xl[x][i];
  // trim trailing no-ops
  while (!flat.empty() && flat.back().kind == K_NOP) flat.pop_back();

  // every index the block kernel derives from an item must stay inside the
  // buffers allocated for this plan
  for (const Item& it : flat) {
    if (it.kind == K_NOP) continue;
    if (it.kind != K_MAC0 || it.tier != 0) return RTA_E_STATE;
    if (it.group < 0 || it.group >= (int)groups.size()) return RTA_E_STATE;
    const Group& gr = groups[it.group];
    if (it.q < 0 || it.q >= c->Q) return RTA_E_STATE;
    if (it.p0 < 0 || it.p1 < it.p0 || it.p1 > T.K) return RTA_E_STATE;
    if (it.k0 < 0 || it.k0 % W != 0 || it.k0 + W > P) return RTA_E_STATE;
    if (it.slot < gr.slot0 || it.slot >= gr.slot0 + gr.nslot || it.slot >= T.nslots) return RTA_E_STATE;
    if (it.target < 1) return RTA_E_STATE;
    if (gr.l0 < 0 || gr.nl < 1 || gr.nl > G || gr.l0 + gr.nl > c->L) return RTA_E_STATE;
  }
  return RTA_OK;
}

KArgs make_args(const rta_ctx* c, const float* in, float* out) {
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
  }
  a.items = c->items;
  a.phase_count = c->phase_count;
  a.groups = c->groups;
  a.state = c->state;
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
  return a;
}

// The two launches of one block, in stream order.
void enqueue_block(const rta_ctx* c, const float* in, float* out, hipStream_t s) {
  const KArgs a = make_args(c, in, out);
  hipLaunchKernelGGL(mac_kernel(c->dtype, c->G), dim3(c->grid), dim3(kThreads), c->lds_bytes, s, a);
  hipLaunchKernelGGL(final_kernel(c->G), dim3(c->n_groups), dim3(kThreads), c->lds_final_bytes, s, a);
}

constexpr size_t kMaxTimedBlocks = 65536;

int launch_block(rta_ctx* c, const float* in, float* out, hipStream_t s) {
  if (c->timing && c->events_used + 3 <= 3 * kMaxTimedBlocks) {
    while (c->events.size() < c->events_used + 3) {
      hipEvent_t e;
      HIP_TRY(c, hipEventCreate(&e));
      c->events.push_back(e);
    }
    hipEvent_t* e = &c->events[c->events_used];
    c->events_used += 3;
    const KArgs a = make_args(c, in, out);
    HIP_TRY(c, hipEventRecord(e[0], s));
    hipLaunchKernelGGL(mac_kernel(c->dtype, c->G), dim3(c->grid), dim3(kThreads), c->lds_bytes, s, a);
    HIP_TRY(c, hipEventRecord(e[1], s));
    hipLaunchKernelGGL(final_kernel(c->G), dim3(c->n_groups), dim3(kThreads), c->lds_final_bytes, s, a);
    HIP_TRY(c, hipEventRecord(e[2], s));
  } else {
    enqueue_block(c, in, out, s);
  }
  HIP_TRY(c, hipGetLastError());
  return RTA_OK;
}

int zero_state(rta_ctx* c) {
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    HIP_TRY(c, hipMemsetAsync(T.X, 0, sizeof(float2) * (size_t)c->Q * T.K * T.P, c->stream));
    if (T.oring)
      HIP_TRY(c, hipMemsetAsync(T.oring, 0, sizeof(float) * (size_t)c->L * c->ring_len, c->stream));
  }
  HIP_TRY(c, hipMemsetAsync(c->hist, 0, sizeof(float) * (size_t)c->Q * c->hist_len, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->state, 0, sizeof(DevState), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
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
  int64_t max_len = 0;
  for (int64_t i = 0; i < (int64_t)c->Q * c->L; ++i) max_len = std::max(max_len, lengths[i]);
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
    c->spectra_bytes += rows * T.P * (int64_t)eb;
    c->h_bytes += (double)rows * T.P * eb;
    c->cmacs += (double)rows * T.P;
    c->x_bytes += (double)c->Q * kmax * T.P * 8.0;
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
  c->ring_len = 1;

  // spectra
  if ((st = build_spectra(c, filters, lengths)) != RTA_OK) return st;

  // work lists
  std::vector<Item> flat;
  std::vector<Group> groups;
  if ((st = build_plan(c, flat, groups)) != RTA_OK) return st;
  c->n_phase = 1;
  c->max_items = (int)std::max<size_t>(1, flat.size());
  c->grid = c->max_items;
  const int32_t pc = (int32_t)flat.size();
  if ((st = dev_alloc(c, &c->items, (size_t)c->max_items)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->phase_count, 1)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->groups, groups.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->state, 1)) != RTA_OK) return st;
  if (!flat.empty())
    HIP_TRY(c, hipMemcpy(c->items, flat.data(), sizeof(Item) * flat.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->phase_count, &pc, sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->groups, groups.data(), sizeof(Group) * groups.size(), hipMemcpyHostToDevice));

  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    if ((st = dev_alloc(c, &T.partial, (size_t)std::max(1, T.nslots) * c->G * T.P)) != RTA_OK) return st;
  }
  if ((st = dev_alloc(c, &c->hist, (size_t)c->Q * c->hist_len)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->d_in, (size_t)c->Q * c->B)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->d_out, (size_t)c->L * c->B)) != RTA_OK) return st;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_in), sizeof(float) * (size_t)c->Q * c->B, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_out), sizeof(float) * (size_t)c->L * c->B, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return RTA_E_NOMEM;
  }

  const int C = vec_bins(c->dtype);
  size_t lds = 0;
  for (int t = 0; t < c->n_tiers; ++t) lds = std::max(lds, sizeof(float2) * 2 * (size_t)c->tier[t].P);
  lds = std::max(lds, sizeof(float2) * (size_t)kThreads * C * c->G);
  c->lds_bytes = lds;
  c->lds_final_bytes = sizeof(float2) * 2 * (size_t)c->tier[0].P;
  int max_lds = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  if ((int64_t)std::max(c->lds_bytes, c->lds_final_bytes) + 64 > (int64_t)max_lds)
    return RTA_E_UNSUPPORTED;
  if (c->lds_bytes > 65536)
    HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(mac_kernel(c->dtype, c->G)),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_bytes));
  if (c->lds_final_bytes > 65536)
    HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(final_kernel(c->G)),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)c->lds_final_bytes));

  return zero_state(c);
}

void free_all(rta_ctx* c) {
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void* p : c->dev_allocs) (void)hipFree(p);
  c->dev_allocs.clear();
  if (c->h_in) (void)hipHostFree(c->h_in);
  if (c->h_out) (void)hipHostFree(c->h_out);
  if (c->stream) (void)hipStreamDestroy(c->stream);
}

int capture_graph(rta_ctx* c) {
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  (void)hipMemcpyAsync(c->d_in, c->h_in, sizeof(float) * (size_t)c->Q * c->B,
                       hipMemcpyHostToDevice, c->stream);
  enqueue_block(c, c->d_in, c->d_out, c->stream);
  (void)hipMemcpyAsync(c->h_out, c->d_out, sizeof(float) * (size_t)c->L * c->B,
                       hipMemcpyDeviceToHost, c->stream);
  HIP_TRY(c, hipStreamEndCapture(c->stream, &c->graph));
  HIP_TRY(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  return RTA_OK;
}

}  // namespace

extern "C" {

int rta_create(rta_ctx** out, double fs, int32_t block, const rta_scheme* scheme, int32_t n_in,
               int32_t n_out, const float* const* filters, const int64_t* lengths,
               int32_t spectra, uint32_t flags) {
  if (out == nullptr) return RTA_E_ARG;
  *out = nullptr;
  std::vector<int> size, count;
  int st = validate(fs, block, scheme, n_in, n_out, filters, lengths, spectra, flags, size, count);
  if (st != RTA_OK) return st;
  rta_ctx* c = new (std::nothrow) rta_ctx();
  if (c == nullptr) return RTA_E_NOMEM;
  c->fs = fs;
  c->B = block;
  c->Q = n_in;
  c->L = n_out;
  c->dtype = spectra;
  c->flags = flags;
  c->G = env_int("RTA_G", 1);
  if (c->G != 1 && c->G != 2 && c->G != 4) c->G = 1;
  c->rows_per_item = env_int("RTA_ROWS", 0);
  st = create_impl(c, size, count, filters, lengths);
  if (st == RTA_OK && !(flags & RTA_FLAG_NO_GRAPH)) st = capture_graph(c);
  if (st != RTA_OK) {
    free_all(c);
    delete c;
    return st;
  }
  *out = c;
  return RTA_OK;
}

int rta_process(rta_ctx* c, const float* in, float* out) {
  if (c == nullptr || in == nullptr || out == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  std::memcpy(c->h_in, in, sizeof(float) * (size_t)c->Q * c->B);
  if (c->flags & RTA_FLAG_NO_GRAPH) {
    HIP_TRY(c, hipMemcpyAsync(c->d_in, c->h_in, sizeof(float) * (size_t)c->Q * c->B,
                              hipMemcpyHostToDevice, c->stream));
    int st = launch_block(c, c->d_in, c->d_out, c->stream);
    if (st != RTA_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->h_out, c->d_out, sizeof(float) * (size_t)c->L * c->B,
                              hipMemcpyDeviceToHost, c->stream));
  } else {
    if (c->gexec == nullptr) return RTA_E_STATE;
    HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
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
  info->spectra_bytes = c->spectra_bytes;
  info->device_bytes = c->device_bytes;
  info->h_bytes_per_block = c->h_bytes;
  info->x_bytes_per_block = c->x_bytes;
  info->io_bytes_per_block = c->io_bytes;
  info->cmacs_per_block = c->cmacs;
  info->grid = c->grid;
  info->outputs_per_group = c->G;
  info->rows_per_item = c->rows_per_item;
  info->poisoned = c->poisoned ? 1 : 0;
  if (c->poisoned) return RTA_E_DEVICE;
  HIP_TRY(c, hipDeviceSynchronize());
  DevState s{};
  HIP_TRY(c, hipMemcpy(&s, c->state, sizeof(s), hipMemcpyDeviceToHost));
  info->blocks_done = s.block;
  return RTA_OK;
}

int rta_timing_enable(rta_ctx* c, int32_t on) {
  if (c == nullptr) return RTA_E_ARG;
  c->timing = on != 0;
  return RTA_OK;
}

int rta_timing_read(rta_ctx* c, int64_t* blocks, double* mac_ms, double* final_ms) {
  if (c == nullptr || blocks == nullptr || mac_ms == nullptr || final_ms == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  *blocks = 0;
  *mac_ms = *final_ms = 0.0;
  for (size_t i = 0; i + 3 <= c->events_used; i += 3) {
    float a = 0.f, b = 0.f;
    HIP_TRY(c, hipEventSynchronize(c->events[i + 2]));
    HIP_TRY(c, hipEventElapsedTime(&a, c->events[i], c->events[i + 1]));
    HIP_TRY(c, hipEventElapsedTime(&b, c->events[i + 1], c->events[i + 2]));
    *mac_ms += a;
    *final_ms += b;
    *blocks += 1;
  }
  c->events_used = 0;
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
