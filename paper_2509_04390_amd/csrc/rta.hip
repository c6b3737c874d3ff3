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
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rta.h"
#include "arena.hpp"
#include "kernels.hpp"

using namespace rta;

namespace {

constexpr int kMinBlock = 16;
constexpr int kMaxBlock = 4096;
constexpr int kXcds = 8;                     // MI355X: 8 XCDs, workgroups round-robin
constexpr int64_t kStageBytes = 64ll << 20;  // filter taps staged per spectra batch
constexpr size_t kMaxTimedBlocks = 65536;

// Scratch of rta_serve_admit_noalloc: the staging of one admission's filter
// spectra build -- an FP16 range flag, the row table and the staged taps --
// in a file-scope device array instead of buffers the library allocates.
// Each device holds its own copy from module load until the process ends.
constexpr int64_t kScratchRows = int64_t(1) << 16;         // spectrum rows per batch
constexpr int64_t kScratchTaps = int64_t(1) << 20;         // staged taps per batch
constexpr size_t kScratchRowsOff = 256;                    // after the range flag
constexpr size_t kScratchTapsOff = kScratchRowsOff + (size_t)kScratchRows * 24;  // SpecRow: 24 B
constexpr size_t kScratchBytes = kScratchTapsOff + (size_t)kScratchTaps * sizeof(float);
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

static_assert(sizeof(SpecRow) == 24, "scratch layout assumes 24-byte rows");
static_assert(kScratchRowsOff % 256 == 0 && kScratchTapsOff % 256 == 0, "scratch alignment");

// Device address of `scratch` on each device (the array's host-side name is
// not a device address), found once per device at set-up; uses of the array
// by overlapping calls in this process are serialized per device.
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_use[kMaxDevices];

// With `dev` current: look up (once) and return the device address of the
// scratch array on `dev`, or nullptr if the runtime refuses.
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}


struct TierHost {
  int P = 0, logP = 0, K = 0, count = 0;
  int kcap = 0;  // serving: partitions of a max_taps filter in this tier
  int64_t offset = 0;
  void* H = nullptr;
  int64_t* pair_row = nullptr;
  int32_t* pair_K = nullptr;
  float2* X = nullptr;
  float2* partial = nullptr;
  float2* tw = nullptr;
  float* oring = nullptr;
  int span = 0;              // filter taps per partition (P, or B when r3)
  int r3 = 0;                // n_f = 3B first tier: P = 3B/2 bins, 3B-point transforms
  float2* tfwd = nullptr;    // tiers >= 1: transform scratch [Q][P] and [L][P]
  float2* tinv = nullptr;
  int nslots = 0;
  int64_t h_rows = 0;        // spectrum rows allocated in H
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

struct Serve;

struct rta_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  double fs = 0;
  int B = 0, Q = 0, L = 0, dtype = 0;
  uint32_t flags = 0;
  int n_tiers = 0;
  TierHost tier[kMaxTiers];
  int G = 1, rows_per_item = 0, n_phase = 1, max_items = 0, n_items = 0;
  int tail_items = 512, tier_rows = 16;
  int max_group_slots = 0;     // first tier: the most partial slots of one output group
  int spectra_loads = 0;       // 0 default, 1 non-temporal, 2 ordinary
  bool nt = true;              // non-temporal spectra loads
  int bin_slices = 0;          // first-tier bin slices per partition row (0: chosen by the plan)
  int n_groups = 0, head_slots = 0, head_nq = 1;
  int64_t hist_len = 0, ring_len = 0;
  size_t lds = 0;              // k_block dynamic LDS
  size_t lds_fused = 0;        // with the feedback convolution in the launch
  int64_t block = 0;           // index of the next block

  void* H01 = nullptr;         // [L][Q][2][P] partitions 0 and 1
  Item* tier_items = nullptr;  // later tiers' transform passes [n_phase][max_tier_items]
  int32_t* tier_count = nullptr;
  int32_t* tier_slot0 = nullptr;
  int32_t* tier_nslot = nullptr;
  int max_tier_items = 0;
  std::vector<int32_t> tier_count_host;  // transform items per phase
  float* hist = nullptr;
  Item* items = nullptr;
  int32_t* phase_count = nullptr;
  Group* groups = nullptr;
  unsigned int* head_count = nullptr;
  unsigned int* heads_done = nullptr;  // heads finished, all blocks (monotonic)
  struct HostStages {          // rta_process host-side timing since create / reset
    int64_t calls = 0, slowest_call = -1, late = 0;
    double max_us[4] = {0, 0, 0, 0}, sum_us[4] = {0, 0, 0, 0}, slowest_us = 0;
  } hs;
  int64_t* n_dev = nullptr;    // graph replay: device block counter
  int64_t n_dev_value = -1;    // what it holds once enqueued work is done (-1: unknown)
  int64_t config_gen = 0;      // bumped when the launch configuration changes

  float* h_in = nullptr;       // pinned host staging, mapped into the device
  float* h_out = nullptr;
  int64_t* h_flag = nullptr;
  int32_t* h_status = nullptr; // pinned error word the kernels may set
  float* m_in = nullptr;       // device addresses of the four
  float* m_out = nullptr;
  int64_t* m_flag = nullptr;
  int32_t* m_status = nullptr;

  rta_ctx* fc = nullptr;        // feedback convolution: outputs -> inputs
  float* d_y = nullptr;         // [L][B] copy of the output block (its input)
  float* d_c = nullptr;         // [Q][B] its output, subtracted next block
  bool fc_fused = false;        // it runs inside this context's launch
  unsigned int* fc_done = nullptr;  // its heads done (fused; monotonic)
  int fc_wait_polls = 1 << 24;  // bound of the synthesis heads' wait for it
  uint32_t fc_wait_bias = 0;    // nonzero only to test the give-up path
  int min_ring = 1;             // first tier's delay line has at least this many slots

  std::vector<int32_t> block_count_host;  // k_block items per phase (active list)
  const int32_t* live = nullptr;  // serving: [Q] live mask of the active list
  int grid_items = 0;             // tail part of the grid
  Serve* serve = nullptr;         // serving state (rta_serve_create)

  bool poisoned = false;
  int timing = 0;                  // timed spans of this many blocks (0: off)
  int64_t timing_base = 0;         // block index at rta_timing_enable
  bool span_open = false;          // a span's first event is recorded
  int timing_span_read = 1;        // blocks per recorded span
  std::vector<hipEvent_t> events;  // 2 per timed block
  size_t events_used = 0;
  int64_t device_bytes = 0, spectra_bytes = 0;
  double h_bytes = 0, x_bytes = 0, io_bytes = 0, cmacs = 0, tail_bytes = 0;
  std::vector<void*> dev_allocs;
};

// Serving state (rta_serve_*; the protocol is described in include/rta.h).
struct ServeSlot {
  int state = RTA_SLOT_FREE;
  bool rows_held = false;  // arena rows not yet returned
  int64_t start = -1, stop = -1, free_at = -1, taps = 0;
  double hb = 0, xb = 0, cm = 0;           // per-block figures of the source
  std::vector<int64_t> row[kMaxTiers];     // [l] first arena row, -1 = none
  std::vector<int32_t> kp[kMaxTiers];      // [l] partitions
};

struct PlanDev {  // one of the two work-list buffers
  Item* items = nullptr;
  int32_t* phase_count = nullptr;
  Item* tier_items = nullptr;
  int32_t* tier_count = nullptr;
  int64_t* pair_row[kMaxTiers] = {};
  int32_t* pair_K[kMaxTiers] = {};
  int32_t* live = nullptr;
  std::vector<int32_t> tier_count_host, block_count_host;
  int grid_items = 0;
  double hb = 0, xb = 0, cm = 0, tb = 0;
};

struct Serve {
  rta_serve_config cfg{};
  std::vector<ServeSlot> slots;
  rta::RowArena arena[kMaxTiers];
  PlanDev dev[2];
  int active = 0;        // buffer the next launch uses
  bool pending = false;  // the other buffer holds a newer list
  hipEvent_t retire[2] = {nullptr, nullptr};
  bool retire_valid[2] = {false, false};
  hipStream_t aux = nullptr;  // spectra and list uploads
  float* d_stage = nullptr;
  int64_t stage_floats = 0;
  SpecRow* d_rows = nullptr;
  int64_t row_cap = 0;
  int* d_range = nullptr;
  std::mutex mu;   // slot states, active/pending; held briefly
  std::mutex ctl;  // serializes admit, release and reset
  int64_t admitted = 0, rej_slots = 0, rej_mem = 0, rej_budget = 0, swaps = 0;
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

// A kernel that could not complete its work correctly (a bounded wait that
// gave up) has set the context's error word: poison the context.
int device_status(rta_ctx* c) {
  if (c->h_status != nullptr && __atomic_load_n(c->h_status, __ATOMIC_ACQUIRE) != 0) {
    c->poisoned = true;
    return RTA_E_DEVICE;
  }
  return RTA_OK;
}

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
int vec_bins(int) { return 2; }  // bins per lane and row in the multiply-accumulate (HVec<>::C)

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

// nt: stream the spectra with non-temporal loads (working sets larger than
// the Infinity Cache) or with ordinary loads (smaller ones, which it can keep
// between blocks)
BlockKernel block_kernel(int dtype, int G, bool nt) {
#define RTA_PICK(HT)                                                   \
  switch (G) {                                                         \
    case 1: return nt ? k_block<HT, 1, true> : k_block<HT, 1, false>;  \
    case 2: return nt ? k_block<HT, 2, true> : k_block<HT, 2, false>;  \
    case 4: return nt ? k_block<HT, 4, true> : k_block<HT, 4, false>;  \
    default: return nullptr;                                           \
  }
  if (dtype == RTA_FP32) RTA_PICK(float2)
  if (dtype == RTA_FP16) RTA_PICK(f16c_t)
  if (dtype == RTA_BF16) RTA_PICK(bf16c_t)
#undef RTA_PICK
  return nullptr;
}

hipError_t launch_spectra(int dtype, dim3 grid, size_t lds, hipStream_t s, const float* taps,
                          const SpecRow* rows, void* H, int P, int logP, int r3, const float2* tw,
                          int* range) {
  if (dtype == RTA_FP32)
    hipLaunchKernelGGL(k_spectra<float2>, grid, dim3(kThreads), lds, s, taps, rows,
                       static_cast<float2*>(H), P, logP, r3, tw, range);
  else if (dtype == RTA_FP16)
    hipLaunchKernelGGL(k_spectra<f16c_t>, grid, dim3(kThreads), lds, s, taps, rows,
                       static_cast<f16c_t*>(H), P, logP, r3, tw, range);
  else
    hipLaunchKernelGGL(k_spectra<bf16c_t>, grid, dim3(kThreads), lds, s, taps, rows,
                       static_cast<bf16c_t*>(H), P, logP, r3, tw, range);
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
  if (flags & ~(RTA_FLAG_SPIKE | RTA_FLAG_NF3)) return RTA_E_ARG;
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
  if ((flags & RTA_FLAG_NF3) && T != 1) return RTA_E_ARG;  // uniform partitions only
  int64_t off = 0;
  for (int t = 0; t < T; ++t) {
    if (!is_pow2(size[t]) || size[t] % block != 0 || size[t] > (1 << 13)) return RTA_E_ARG;
    if (t > 0 && size[t] <= size[t - 1]) return RTA_E_ARG;
    if (count[t] < 0 || (count[t] == 0 && t != T - 1)) return RTA_E_ARG;
    // a later tier's frame needs two blocks for its transform, at least one
    // for its multiply-accumulate and two for its inverse transform before
    // its first output sample is due (o_t >= P_t + 4B)
    if (t > 0 && off < (int64_t)size[t] + 4 * (int64_t)block) return RTA_E_ARG;
    off += (int64_t)count[t] * size[t];
  }
  if (count[T - 1] > 0 && max_len > off) return RTA_E_ARG;
  return RTA_OK;
}

// ---------------------------------------------------------------------------
// Work lists.  The block index n selects phase n mod n_phase (n_phase =
// P_max / B).  The tail list of a phase holds
//   - the first tier's tail items (every phase): partitions p >= 2 of every
//     (output group, input), cut into chunks of about R rows and bin slices;
//     each chunk owns one partial slot of its group (the heads do p = 0, 1);
//   - the multiply-accumulate items of later tiers whose frame is being
//     accumulated in that block.
// The transform list of a phase holds the later tiers' transform passes
// (kernels.hpp, "Later tiers"): for a frame whose input completes in block
// n_f, K_FFT_A in n_f, K_FFT_B in n_f + 1, its multiply-accumulate in
// n_f + 2 .. n_f + nmac + 1, K_FIN_A in n_f + nmac + 2 and K_FIN_B in
// n_f + nmac + 3.  Tier t (P_t = r B, offset o_t) leaves s = (o_t + B - P_t)
// / B blocks between input completion and first output, so nmac <= s - 4;
// the next frame's K_FFT_B (block n_f + r + 1) overwrites the ring slot that
// this frame's last partition reads, so nmac <= r - 1.  nmac = min(s - 4,
// r - 1), or 1 with RTA_FLAG_SPIKE.
// ---------------------------------------------------------------------------
struct Bucket {
  int tier, q, p0, k0;
  std::vector<Item> items;
  int64_t rows = 0;
};

struct Plan {
  std::vector<std::vector<Item>> block;  // per phase: tail items
  std::vector<std::vector<Item>> tier;   // per phase: transform passes
  std::vector<Group> groups;
  std::vector<int32_t> tier_slot0, tier_nslot;  // [tier][group]
};

// nmac of tier t >= 1 (see above)
int tier_nmac(const rta_ctx* c, int t) {
  const TierHost& T = c->tier[t];
  const int r = T.P / c->B;
  const int64_t s = (T.offset + c->B - T.P) / c->B;
  if (c->flags & RTA_FLAG_SPIKE) return 1;
  return (int)std::min<int64_t>(s - 4, r - 1);
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

// A bucket holds every bin slice of one partition range (all of each row's
// bytes): an XCD that streamed only one byte range of every row would reach
// only part of the HBM channels (measured: the XCDs holding one slice of two
// finished 3 us after the others).
void add_to_bucket(std::vector<Bucket>& buckets, const Item& it, int nl) {
  auto bit = std::find_if(buckets.begin(), buckets.end(), [&](const Bucket& b) {
    return b.tier == it.tier && b.q == it.q && b.p0 == it.p0;
  });
  if (bit == buckets.end()) {
    buckets.push_back(Bucket{it.tier, it.q, it.p0, 0, {}, 0});
    bit = buckets.end() - 1;
  }
  bit->items.push_back(it);
  bit->rows += (int64_t)(it.p1 - it.p0) * nl;
}

int build_plan(rta_ctx* c, Plan& plan) {
  const int G = c->G;
  const int C = vec_bins(c->dtype);
  const int ngroups = (c->L + G - 1) / G;
  const bool fixed = c->serve != nullptr;
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
  // a multiply-accumulate item's per-output spectrum rows (Item::row, pend)
  auto mac_rows = [&](Item& it, const TierHost& T) {
    const Group& gr = plan.groups[it.group];
    it.nl = gr.nl;
    for (int g = 0; g < 4; ++g) {
      it.pend[g] = 0;
      it.row[g] = 0;
    }
    for (int g = 0; g < gr.nl; ++g) {
      const size_t pair = (size_t)(gr.l0 + g) * c->Q + it.q;
      if (T.row[pair] >= 0) {
        it.row[g] = T.row[pair];
        it.pend[g] = std::min(it.p1, T.kp[pair]);
      }
    }
  };

  // ---- first tier: partitions >= 2, every phase
  std::vector<Item> tier0;
  {
    TierHost& T = c->tier[0];
    // bin slices per row: each item covers W bins of nslice-fold more rows,
    // so an output group owns nslice-fold fewer partial slots for the heads
    // to reduce; a wave still reads whole 16-byte-per-lane segments of
    // 64 / (W / C) rows
    // (a power of two dividing P: with n_f = 3B, P = 3B/2 gives thirds)
    const int Wmax = std::min(T.r3 ? T.P / 3 : T.P, kThreads * C);
    int W = std::max(C, Wmax / std::max(1, c->bin_slices)), nslice = T.P / W;
    int64_t total_rows = 0;
    for (const Group& gr : plan.groups)
      for (int q = 0; q < c->Q; ++q) total_rows += std::max(0, group_rows(T, gr, q) - 2);
    // serving: every (group, input) owns the slots of a max_taps filter, so
    // a slot's meaning does not depend on which sources are present
    const int cap_rows = fixed ? std::max(0, T.kcap - 2) : 0;
    if (fixed) total_rows = (int64_t)ngroups * c->Q * cap_rows;
    int R = c->rows_per_item;
    if (R <= 0) {
      const int64_t target_items = std::max(1, c->tail_items);
      R = (int)std::max<int64_t>(8, (total_rows * nslice + target_items - 1) / target_items);
      // Slots per output group within what a head adds up from registers
      // while it transforms its window (HeadRed: 16 slots per thread, 256 / P
      // threads per bin): with few outputs and long filters the item count
      // above would give one group hundreds of slots, and its head would
      // reduce them after the transform.  Rows per item grow to the cap; with
      // automatic slices, narrower bin ranges then cut the items back to
      // about 32 KB of rows each (one workgroup streams some 10-15 GB/s, so
      // an item's share stays within a few microseconds).
      int Rmin = 8;
      const int ng = T.P <= kThreads ? kThreads / T.P : 0;
      if (!fixed && !T.r3 && ng > 0 && is_pow2(T.P) &&
          (c->Q + ng - 1) / ng <= HeadRed<float2>::kInputs) {
        const int cap = HeadRed<float2>::kSlots * ng;
        auto ranges = [&](int r, bool worst) {  // slots of the fullest group, or all ranges
          int64_t tot = 0, m = 0;
          for (const Group& gr : plan.groups) {
            int64_t ns = 0;
            for (int q = 0; q < c->Q; ++q) ns += (std::max(0, group_rows(T, gr, q) - 2) + r - 1) / r;
            tot += ns;
            m = std::max(m, ns);
          }
          return worst ? m : tot;
        };
        if (ranges(R, true) > cap) {
          int rc = R;
          while (ranges(rc, true) > cap) rc = std::max(rc + 1, rc + rc / 16);
          while (rc > R && ranges(rc - 1, true) <= cap) --rc;  // the smallest that fits
          if (c->bin_slices == 0)
            while (ranges(rc, false) * nslice < target_items && W / 2 >= C && T.P % (W / 2) == 0 &&
                   total_rows * T.P * 8 / (ranges(rc, false) * nslice) > (32 << 10)) {
              W /= 2;
              nslice *= 2;
            }
          R = (int)std::max<int64_t>(rc, (total_rows * nslice + target_items - 1) / target_items);
          Rmin = rc;
        }
      }
      // XCD balance: the partition ranges of one input form one bucket per
      // range (all groups, all slices), spread over the 8 XCDs; make the
      // number of ranges of the longest (group, input) times the inputs a
      // multiple of 8 so every XCD gets as many (measured, 1 -> 32 x 10 s:
      // 60 ranges 27.5 us, 64 ranges 24.4 us)
      int kmax = 0;
      for (const Group& gr : plan.groups)
        for (int q = 0; q < c->Q; ++q) kmax = std::max(kmax, group_rows(T, gr, q) - 2);
      if (fixed) kmax = std::max(0, T.kcap - 2);
      int step = kXcds;
      for (int qq = c->Q; qq % 2 == 0 && step > 1; qq /= 2) step /= 2;  // 8 / gcd(Q, 8)
      if ((kmax + R - 1) / R >= kXcds)  // the largest R' <= R giving a multiple of step
        for (int r2 = R; r2 >= Rmin; --r2)
          if (((kmax + r2 - 1) / r2) % step == 0) {
            R = r2;
            break;
          }
    }
    c->rows_per_item = R;
    if (c->bin_slices == 0) c->bin_slices = Wmax / W;  // later plans keep this layout
    const int nch_cap = (cap_rows + R - 1) / R;
    int slot = 0;
    for (int g = 0; g < ngroups; ++g) {
      Group& gr = plan.groups[g];
      gr.slot0 = slot;
      gr.nslot = 0;
      if (fixed) {
        gr.nslot = c->Q * nch_cap;
        slot += gr.nslot;
      }
      for (int q = 0; q < c->Q; ++q) {
        const int kg = group_rows(T, gr, q);
        if (kg <= 2) continue;  // partitions 0 and 1 are done by the heads
        const int rows = kg - 2;
        const int nch = (rows + R - 1) / R;
        for (int ch = 0; ch < nch; ++ch) {
          const int p0 = fixed ? 2 + ch * R : 2 + (int)((int64_t)ch * rows / nch);
          const int p1 = fixed ? std::min(kg, 2 + (ch + 1) * R) : 2 + (int)((int64_t)(ch + 1) * rows / nch);
          const int it_slot = fixed ? gr.slot0 + q * nch_cap + ch : slot;
          for (int sl = 0; sl < nslice; ++sl) {
            Item it{};
            it.kind = K_MAC;
            it.tier = 0;
            it.group = g;
            it.q = q;
            it.p0 = p0;
            it.p1 = p1;
            it.k0 = sl * W;
            it.w = W;
            it.slot = it_slot;
            mac_rows(it, T);
            tier0.push_back(it);
          }
          if (!fixed) {
            ++slot;
            ++gr.nslot;
          }
        }
      }
    }
    T.nslots = slot;
    c->max_group_slots = 0;
    for (const Group& gr : plan.groups) c->max_group_slots = std::max(c->max_group_slots, gr.nslot);
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
    struct Chunk { int g, q, p0, p1, slot, cap, acc; };
    std::vector<Chunk> chunks;
    const int nch_cap = fixed ? (T.kcap + R - 1) / R : 0;
    for (int g = 0; g < ngroups; ++g)
      for (int q = 0; q < c->Q; ++q) {
        const int kg = group_rows(T, plan.groups[g], q);
        if (kg == 0) continue;
        const int nch = (kg + R - 1) / R;
        for (int ch = 0; ch < nch; ++ch) {
          if (fixed)
            chunks.push_back(Chunk{g, q, ch * R, std::min(kg, (ch + 1) * R), 0,
                                   (g * c->Q + q) * nch_cap + ch, 0});
          else
            chunks.push_back(Chunk{g, q, (int)((int64_t)ch * kg / nch),
                                   (int)((int64_t)(ch + 1) * kg / nch), 0, 0, 0});
        }
      }
    // spread the chunks over the nmac blocks, balancing rows (the block of a
    // chunk never decreases along a (group, input)'s partitions); with the
    // fixed serving layout a chunk's block depends on its capacity index
    // alone, so work lists of any set of sources agree on it
    int64_t total = 0;
    for (const Chunk& ch : chunks) total += ch.p1 - ch.p0;
    std::vector<int> when(chunks.size(), 0);
    int64_t acc = 0;
    const int64_t ncap = (int64_t)ngroups * c->Q * nch_cap;
    auto cap_when = [&](int64_t cap) {
      return (int)std::min<int64_t>(nmac - 1, cap * nmac / std::max<int64_t>(1, ncap));
    };
    for (size_t i = 0; i < chunks.size(); ++i) {
      when[i] = fixed ? cap_when(chunks[i].cap)
                      : (total > 0 ? (int)std::min<int64_t>(nmac - 1, acc * nmac / total) : 0);
      acc += chunks[i].p1 - chunks[i].p0;
    }
    // partial slots: chunks of one (group, input) accumulated in different
    // blocks share a slot -- the first in frame order stores, the later ones
    // add -- so a group owns only as many slots per input as it has chunks in
    // one block, and its final step has that few to reduce.  rank = chunks of
    // the same (group, input) and block before this one.
    // for a (group, input)'s chunks in partition order (blocks w[] non-
    // decreasing): rank[ch] within its block, acc[ch] = an earlier block had
    // a chunk of the same rank; returns the slots needed
    auto rank_chunks = [](const std::vector<int>& w, std::vector<int>& rank, std::vector<int>& accf) {
      const int n = (int)w.size();
      rank.assign(n, 0);
      accf.assign(n, 0);
      int before = 0, in_block = 0, slots = 0;  // widest earlier block, this block so far
      for (int ch = 0; ch < n; ++ch) {
        if (ch > 0 && w[ch] != w[ch - 1]) {
          before = std::max(before, in_block);
          in_block = 0;
        }
        rank[ch] = in_block++;
        accf[ch] = rank[ch] < before ? 1 : 0;
        slots = std::max(slots, rank[ch] + 1);
      }
      return slots;
    };
    std::vector<int> wcap, rk, af;
    int nsl_cap = 0;
    if (fixed)  // a present source's chunks are a prefix of the capacity chunks
      for (int g = 0; g < ngroups; ++g)
        for (int q = 0; q < c->Q; ++q) {
          wcap.assign(nch_cap, 0);
          for (int ch = 0; ch < nch_cap; ++ch) wcap[ch] = cap_when((int64_t)(g * c->Q + q) * nch_cap + ch);
          nsl_cap = std::max(nsl_cap, rank_chunks(wcap, rk, af));
        }
    int slot = 0;
    size_t i0 = 0;
    for (int g = 0; g < ngroups; ++g) {
      plan.tier_slot0[(size_t)t * ngroups + g] = slot;
      const int gslot0 = slot;
      if (fixed) slot += c->Q * nsl_cap;
      for (int q = 0; q < c->Q; ++q) {
        size_t i1 = i0;
        while (i1 < chunks.size() && chunks[i1].g == g && chunks[i1].q == q) ++i1;
        std::vector<int> w(when.begin() + i0, when.begin() + i1);
        if (fixed) {
          wcap.assign(nch_cap, 0);
          for (int ch = 0; ch < nch_cap; ++ch) wcap[ch] = cap_when((int64_t)(g * c->Q + q) * nch_cap + ch);
        }
        const int nsl = rank_chunks(fixed ? wcap : w, rk, af);
        for (size_t i = i0; i < i1; ++i) {
          const int ch = (int)(i - i0);
          chunks[i].acc = af[ch];
          chunks[i].slot = fixed ? gslot0 + q * nsl_cap + rk[ch] : slot + rk[ch];
        }
        if (!fixed) slot += nsl;
        i0 = i1;
      }
      plan.tier_nslot[(size_t)t * ngroups + g] = slot - plan.tier_slot0[(size_t)t * ngroups + g];
    }
    T.nslots = slot;
    // transform passes: items of rows (K_FFT_A, K_FIN_B) and of column
    // pairs (K_FFT_B, K_FIN_A)
    const int rpi = tier_rows_per_item(T.logP), ppi = tier_pairs_per_item(T.logP);
    const int N1 = 1 << tier_lg1(T.logP), N2 = T.P / N1;
    auto pass = [&](int kind, int ph0, int lag, int q, int g, int nitems, int w) {
      for (int j = 0; j < nitems; ++j) {
        Item it{};
        it.kind = kind;
        it.tier = t;
        it.q = q;
        it.group = g;
        it.k0 = j;
        it.w = w;
        it.lag = lag;
        plan.tier[(ph0 + lag) % n_phase].push_back(it);
      }
    };
    for (int ph0 = r - 1; ph0 < n_phase; ph0 += r) {  // phases in which a frame completes
      for (int q = 0; q < c->Q; ++q) {
        bool used = false;
        for (int l = 0; l < c->L; ++l) used |= T.kp[l * c->Q + q] > 0;
        if (!used) continue;
        pass(K_FFT_A, ph0, 0, q, 0, N1 / rpi, rpi);
        pass(K_FFT_B, ph0, 1, q, 0, N2 / (2 * ppi), ppi);
      }
      for (size_t i = 0; i < chunks.size(); ++i) {
        const int lag = 2 + when[i];
        for (int sl = 0; sl < nslice; ++sl) {
          Item it{};
          it.kind = K_MAC;
          it.tier = t;
          it.group = chunks[i].g;
          it.q = chunks[i].q;
          it.p0 = chunks[i].p0;
          it.p1 = chunks[i].p1;
          it.k0 = sl * W;
          it.w = W;
          it.slot = chunks[i].slot;
          it.acc = chunks[i].acc;
          it.lag = lag;
          mac_rows(it, T);
          tier_mac[(ph0 + lag) % n_phase].push_back(it);
        }
      }
      for (int g = 0; g < ngroups; ++g) {
        if (plan.tier_nslot[(size_t)t * ngroups + g] == 0) continue;
        if (fixed && chunks.empty()) continue;  // no source present
        for (int gi = 0; gi < plan.groups[g].nl; ++gi) {  // every output of the group
          pass(K_FIN_A, ph0, nmac + 2, gi, g, N2 / (2 * ppi), ppi);
          pass(K_FIN_B, ph0, nmac + 3, gi, g, N1 / rpi, rpi);
        }
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
      const int W = it.w;
      if (it.q < 0 || it.q >= c->Q) return RTA_E_STATE;
      if (it.p0 < (it.tier == 0 ? 2 : 0) || it.p1 < it.p0 || it.p1 > T.K) return RTA_E_STATE;
      if (W < C || W > kThreads * C || (W & (W - 1)) != 0 || T.P % W != 0) return RTA_E_STATE;
      if (it.k0 < 0 || it.k0 % W != 0 || it.k0 + W > T.P) return RTA_E_STATE;
      if (it.nl != plan.groups[it.group].nl) return RTA_E_STATE;
      for (int g = 0; g < it.nl; ++g)
        if (it.pend[g] < 0 || it.pend[g] > it.p1 || it.row[g] < 0 ||
            (it.pend[g] > 0 && it.row[g] + it.pend[g] > T.h_rows))
          return RTA_E_STATE;
      if (it.tier == 0) {
        const Group& gr = plan.groups[it.group];
        if (it.slot < gr.slot0 || it.slot >= gr.slot0 + gr.nslot) return RTA_E_STATE;
      } else {
        const int s0 = plan.tier_slot0[(size_t)it.tier * ngroups + it.group];
        const int ns = plan.tier_nslot[(size_t)it.tier * ngroups + it.group];
        if (it.slot < s0 || it.slot >= s0 + ns) return RTA_E_STATE;
        if (it.lag < 2 || it.lag > tier_nmac(c, it.tier) + 1) return RTA_E_STATE;
      }
    }
    for (const Item& it : plan.tier[ph]) {
      if (it.tier < 1 || it.tier >= c->n_tiers) return RTA_E_STATE;
      const TierHost& T = c->tier[it.tier];
      const int nmac = tier_nmac(c, it.tier);
      const int N1 = 1 << tier_lg1(T.logP), N2 = T.P / N1;
      const int rpi = tier_rows_per_item(T.logP), ppi = tier_pairs_per_item(T.logP);
      const bool rows = it.kind == K_FFT_A || it.kind == K_FIN_B;
      const int w = rows ? rpi : ppi, n = rows ? N1 / rpi : N2 / (2 * ppi);
      if (it.w != w || it.k0 < 0 || it.k0 >= n) return RTA_E_STATE;
      if (rows ? (N1 % rpi != 0 || rpi * N2 > kTierBuf) : (N2 % (2 * ppi) != 0 || 2 * ppi * N1 > kTierBuf))
        return RTA_E_STATE;
      if (N2 > 128 || N1 > N2) return RTA_E_STATE;
      switch (it.kind) {
        case K_FFT_A:
        case K_FFT_B:
          if (it.q < 0 || it.q >= c->Q || it.lag != (it.kind == K_FFT_A ? 0 : 1)) return RTA_E_STATE;
          break;
        case K_FIN_A:
        case K_FIN_B:
          if (it.group < 0 || it.group >= ngroups || it.q < 0 || it.q >= plan.groups[it.group].nl ||
              it.lag != nmac + (it.kind == K_FIN_A ? 2 : 3))
            return RTA_E_STATE;
          break;
        default:
          return RTA_E_STATE;
      }
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
    d.tfwd = T.tfwd;
    d.tinv = T.tinv;
    d.lg1 = tier_lg1(T.logP);
    d.r3 = T.r3;
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
  a.n_head = c->L;
  a.head_slots = c->head_slots;
  a.n = n;
  a.H01 = c->H01;
  a.head_count = c->head_count;
  a.heads_done = c->heads_done;
  a.done_flag = nullptr;  // set by rta_process, which polls it
  a.tier_items = c->tier_items;
  a.tier_count = c->tier_count;
  a.tier_slot0 = c->tier_slot0;
  a.tier_nslot = c->tier_nslot;
  a.max_tier_items = c->max_tier_items;
  a.n_groups_total = c->n_groups;
  a.live = c->live;
  a.status = c->m_status;
  if (c->fc != nullptr && c->fc_fused) {
    const rta_ctx* f = c->fc;
    const TierHost& T = f->tier[0];
    FcArgs& F = a.fc;
    F.T.H = T.H;
    F.T.pair_row = T.pair_row;
    F.T.pair_K = T.pair_K;
    F.T.X = T.X;
    F.T.partial = T.partial;
    F.T.tw = T.tw;
    F.T.oring = nullptr;
    F.T.offset = 0;
    F.T.P = T.P;
    F.T.logP = T.logP;
    F.T.r3 = T.r3;
    F.T.K = T.K;
    F.T.nslots = std::max(1, T.nslots);
    F.T.r = 1;
    F.items = f->items;
    F.groups = f->groups;
    F.H01 = f->H01;
    F.hist = f->hist;
    F.c = c->d_c;
    F.done = c->fc_done;
    F.hist_mask = f->hist_len - 1;
    F.n_items = f->block_count_host.empty() ? 0 : f->block_count_host[0];
    F.tail0 = c->grid_items;
    F.n_heads = f->L;
    F.head_slots = (f->L + kXcds - 1) / kXcds * kXcds;
    F.Qf = f->Q;
    F.Lf = f->L;
    F.wait_polls = c->fc_wait_polls;
    F.wait_bias = c->fc_wait_bias;
    a.fc_on = 1;
    a.nf3 = T.r3;
    a.sub = c->d_c;
  }
  return a;
}

// Make buffer d the one launches read.
void activate(rta_ctx* c, const PlanDev& d) {
  c->items = d.items;
  c->phase_count = d.phase_count;
  c->tier_items = d.tier_items;
  c->tier_count = d.tier_count;
  c->tier_count_host = d.tier_count_host;
  c->block_count_host = d.block_count_host;
  for (int t = 0; t < c->n_tiers; ++t) {
    c->tier[t].pair_row = d.pair_row[t];
    c->tier[t].pair_K = d.pair_K[t];
  }
  c->live = d.live;
  c->grid_items = d.grid_items;
  c->h_bytes = d.hb;
  c->x_bytes = d.xb;
  c->cmacs = d.cm;
  c->tail_bytes = d.tb;
}

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Serving: first block from which a slot whose input stopped at block m owns
// only zeros -- its delay lines of every tier, input history and partial
// sums -- so its work items can be dropped and its rows reused.  Tier t's
// frames f <= f_last see input before m; frame f_last + K_t is the first
// whose delay line is all zero, and its slots are rewritten (with zeros) by
// the time its final step has run.
int64_t drain_end(const rta_ctx* c, int64_t m) {
  int64_t end = m;
  for (int t = 0; t < c->n_tiers; ++t) {
    const TierHost& T = c->tier[t];
    const int64_t P = T.P, r = T.P / c->B;
    const int64_t fl = floor_div(m * c->B - 1, P) + 1;
    const int64_t e = t == 0 ? fl + T.K + 1 : (fl + T.K + 1) * r + tier_nmac(c, t) + 3;
    end = std::max(end, e + 1);
  }
  return end;
}

// Serving: at a block boundary, switch to a newer work list and advance the
// slot states (block thread; short critical section).
int serve_boundary(rta_ctx* c, hipStream_t s) {
  Serve* sv = c->serve;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->pending) {
    // launches so far used the old buffer; this event passes once they are
    // done, after which a control call may overwrite it
    HIP_TRY(c, hipEventRecord(sv->retire[sv->active], s));
    sv->retire_valid[sv->active] = true;
    sv->active ^= 1;
    sv->pending = false;
    ++sv->swaps;
    activate(c, sv->dev[sv->active]);
    for (ServeSlot& sl : sv->slots) {
      if (sl.state == RTA_SLOT_JOINING) {
        sl.state = RTA_SLOT_LIVE;
        sl.start = c->block;
      } else if (sl.state == RTA_SLOT_LEAVING) {
        sl.state = RTA_SLOT_DRAINING;
        sl.stop = c->block;
        sl.free_at = drain_end(c, c->block);
      }
    }
  }
  for (ServeSlot& sl : sv->slots)
    if (sl.state == RTA_SLOT_DRAINING && c->block >= sl.free_at) sl.state = RTA_SLOT_FREE;
  return RTA_OK;
}

// Grid and dynamic LDS of the launch of block n (its phase's transform
// passes); sets a.tier_slots.
void block_geometry(const rta_ctx* c, int64_t n, KArgs& a, unsigned& grid, size_t& lds) {
  const int phase = (int)(n % c->n_phase);
  const int n_tier = c->tier_count_host.empty() ? 0 : c->tier_count_host[phase];
  a.tier_slots = (n_tier + kXcds - 1) / kXcds * kXcds;  // keeps the tails' XCD residues
  grid = (unsigned)(c->head_slots + a.tier_slots + c->grid_items);
  lds = c->lds;
  if (a.fc_on) {
    grid += (unsigned)(a.fc.head_slots + a.fc.n_items);
    lds = c->lds_fused;
  }
}

// One block: heads of block n, the later tiers' transform passes of this
// phase and tails of block n + 1 in a single launch.
// `flag`: raise the host-visible completion flag (rta_process).
int launch_block(rta_ctx* c, const float* in, float* out, hipStream_t s, bool flag = false) {
  if (c->serve != nullptr) {
    const int st = serve_boundary(c, s);
    if (st != RTA_OK) return st;
  }
  KArgs a = make_args(c, in, out, c->block);
  if (flag) {
    a.done_flag = c->m_flag;
    // a real-time block: its output first, when the tails stream enough to
    // slow the heads down (measured: 1 -> 32 x 480,000 taps FP32 paced p50
    // 41 -> 33 us, 1 -> 64 x 576,000 taps 56 -> 41 us; with the 11 MB per
    // block of the 4 -> 64 NUPC workload the waiting tails' polls cost more
    // than they saved)
    a.tails_wait = c->h_bytes >= 32e6 ? 1 : 0;
  }
  unsigned grid = 0;
  size_t lds = 0;
  block_geometry(c, c->block, a, grid, lds);
  // timing: spans of `timing` consecutive blocks, the first starting at the
  // first block launched after rta_timing_enable; an event before a span's
  // first launch and one after its last
  const int64_t every = c->timing;
  const int64_t rel = c->block - c->timing_base;
  const bool span_start = every > 0 && rel % every == 0 && c->events_used + 2 <= 2 * kMaxTimedBlocks;
  const bool span_end = every > 0 && c->span_open && (rel + 1) % every == 0;
  if (span_start) {
    while (c->events.size() < c->events_used + 2) {
      hipEvent_t ev;
      HIP_TRY(c, hipEventCreate(&ev));
      c->events.push_back(ev);
    }
    HIP_TRY(c, hipEventRecord(c->events[c->events_used], s));
    c->span_open = true;
  }
  if (c->fc != nullptr && !c->fc_fused) {
    a.sub = c->d_c;
    a.out2 = c->d_y;
  }
  hipLaunchKernelGGL(block_kernel(c->dtype, c->G, c->nt), dim3(grid), dim3(kThreads), lds, s, a);
  HIP_TRY(c, hipGetLastError());
  if (c->fc != nullptr && c->fc_fused) {
    c->fc->block += 1;  // ran inside this launch
  } else if (c->fc != nullptr) {  // feedback estimate of this block, for the next one
    const int st = launch_block(c->fc, c->d_y, c->d_c, s);
    if (st != RTA_OK) {
      c->poisoned = true;
      return st;
    }
  }
  if (span_end || (span_start && every == 1)) {
    HIP_TRY(c, hipEventRecord(c->events[c->events_used + 1], s));
    c->events_used += 2;
    c->span_open = false;
  }
  c->block += 1;
  return RTA_OK;
}

int zero_state(rta_ctx* c) {
  c->hs = rta_ctx::HostStages{};
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    HIP_TRY(c, hipMemsetAsync(T.X, 0, sizeof(float2) * (size_t)c->Q * T.K * T.P, c->stream));
    // before the first block the terms p >= 2 are all zero (zero history)
    HIP_TRY(c, hipMemsetAsync(T.partial, 0,
                              sizeof(float2) * (t == 0 ? 2 : 1) * (size_t)std::max(1, T.nslots) * c->G * T.P,
                              c->stream));
    if (T.oring)
      HIP_TRY(c, hipMemsetAsync(T.oring, 0, sizeof(float) * (size_t)c->L * c->ring_len, c->stream));
    // the first blocks after a reset run the transform passes of frames
    // before block 0 (all-zero input): their scratch must hold zeros too
    if (T.tfwd) HIP_TRY(c, hipMemsetAsync(T.tfwd, 0, sizeof(float2) * (size_t)c->Q * T.P, c->stream));
    if (T.tinv) HIP_TRY(c, hipMemsetAsync(T.tinv, 0, sizeof(float2) * (size_t)c->L * T.P, c->stream));
  }
  HIP_TRY(c, hipMemsetAsync(c->hist, 0, sizeof(float) * (size_t)c->Q * c->hist_len, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->head_count, 0, sizeof(unsigned int), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->heads_done, 0, sizeof(unsigned int), c->stream));
  if (c->d_c) HIP_TRY(c, hipMemsetAsync(c->d_c, 0, sizeof(float) * (size_t)c->Q * c->B, c->stream));
  if (c->fc_done) HIP_TRY(c, hipMemsetAsync(c->fc_done, 0, sizeof(unsigned int), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->fc) {
    const int st = zero_state(c->fc);
    if (st != RTA_OK) return st;
  }
  __atomic_store_n(c->h_flag, (int64_t)0, __ATOMIC_RELEASE);
  c->block = 0;
  c->timing_base = 0;  // a span still open is dropped
  c->span_open = false;
  return RTA_OK;
}

// Temporary device buffer released when it goes out of scope.
struct TmpDev {
  void* p = nullptr;
  ~TmpDev() {
    if (p) (void)hipFree(p);
  }
};

// One filter's partitions in one tier: taps [o_t, o_t + kp P_t) of `taps`
// (len taps in all) go to spectra rows [row, row + kp).
struct SpecJob {
  int tier;
  const float* taps;
  int64_t len, row;
  int kp;
};

// Build the spectra rows of `jobs` on stream s through the given device
// staging buffers (d_stage: stage_floats taps, at least one whole filter;
// d_rows: row_cap rows, at least stage_floats / P_0 + jobs per tier).
// Synchronous; RTA_E_RANGE when an FP16 spectrum value overflows.
int run_spectra(rta_ctx* c, const std::vector<SpecJob>& jobs, hipStream_t s, float* d_stage,
                int64_t stage_floats, SpecRow* d_rows, int64_t row_cap, int* d_range) {
  HIP_TRY(c, hipMemsetAsync(d_range, 0, sizeof(int), s));
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    const int P = T.P;
    const size_t lds = sizeof(float2) * 2 * (size_t)P;
    std::vector<SpecRow> rows;
    std::vector<float> host_stage;
    auto flush = [&]() -> int {
      if (rows.empty()) return RTA_OK;
      HIP_TRY(c, hipMemcpyAsync(d_stage, host_stage.data(), sizeof(float) * host_stage.size(),
                                hipMemcpyHostToDevice, s));
      HIP_TRY(c, hipMemcpyAsync(d_rows, rows.data(), sizeof(SpecRow) * rows.size(),
                                hipMemcpyHostToDevice, s));
      HIP_TRY(c, launch_spectra(c->dtype, dim3((unsigned)rows.size()), lds, s, d_stage, d_rows, T.H,
                                P, T.logP, T.r3, T.tw, d_range));
      HIP_TRY(c, hipStreamSynchronize(s));
      rows.clear();
      host_stage.clear();
      return RTA_OK;
    };
    int st;
    for (const SpecJob& j : jobs) {
      if (j.tier != t || j.kp == 0) continue;
      const int64_t a0 = T.offset, a1 = std::min(j.len, T.offset + (int64_t)j.kp * T.span);
      const int64_t n = std::max<int64_t>(0, a1 - a0);
      if (n > stage_floats || j.kp > row_cap) return RTA_E_STATE;
      if ((int64_t)host_stage.size() + n > stage_floats || (int64_t)rows.size() + j.kp > row_cap)
        if ((st = flush()) != RTA_OK) return st;
      const int64_t base = (int64_t)host_stage.size();
      if (n > 0) host_stage.insert(host_stage.end(), j.taps + a0, j.taps + a1);
      for (int p = 0; p < j.kp; ++p) {
        SpecRow r{};
        r.src = base + (int64_t)p * T.span;
        r.len = (int32_t)std::max<int64_t>(0, std::min<int64_t>(T.span, n - (int64_t)p * T.span));
        r.dst = j.row + p;
        rows.push_back(r);
      }
    }
    if ((st = flush()) != RTA_OK) return st;
  }
  int range = 0;
  HIP_TRY(c, hipMemcpyAsync(&range, d_range, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return range ? RTA_E_RANGE : RTA_OK;
}

int build_spectra(rta_ctx* c, const float* const* filters, const int64_t* lengths) {
  int64_t max_len = 0;
  for (int64_t i = 0; i < (int64_t)c->Q * c->L; ++i) max_len = std::max(max_len, lengths[i]);
  const int64_t stage_floats = std::max<int64_t>(max_len, kStageBytes / 4);
  // a batch holds at most stage_floats taps, hence at most this many rows
  const int64_t row_cap = stage_floats / c->tier[0].span + (int64_t)c->Q * c->L + 1;
  TmpDev stage, drows, drange;
  if (hipMalloc(&stage.p, sizeof(float) * (size_t)stage_floats) != hipSuccess ||
      hipMalloc(&drows.p, sizeof(SpecRow) * (size_t)row_cap) != hipSuccess ||
      hipMalloc(&drange.p, sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    return RTA_E_NOMEM;
  }
  std::vector<SpecJob> jobs;
  for (int t = 0; t < c->n_tiers; ++t) {
    const TierHost& T = c->tier[t];
    for (int l = 0; l < c->L; ++l)
      for (int q = 0; q < c->Q; ++q) {
        const int pair_in = q * c->L + l;  // caller layout [in][out]
        const int pair = l * c->Q + q;     // device layout [out][in]
        if (T.kp[pair] == 0) continue;
        jobs.push_back(SpecJob{t, filters[pair_in], lengths[pair_in], T.row[pair], T.kp[pair]});
      }
  }
  return run_spectra(c, jobs, c->stream, static_cast<float*>(stage.p), stage_floats,
                     static_cast<SpecRow*>(drows.p), row_cap, static_cast<int*>(drange.p));
}

// ---------------------------------------------------------------------------
// Serving: work-list buffers.
// ---------------------------------------------------------------------------

// Copy `plan`, the pair tables in c->tier[].row/kp and the live mask into
// buffer d on stream s (synchronous).  Lists longer than the buffers' stride
// (the stride is the longest list of the every-slot-present plan) lose their
// XCD padding instead; the items are a subset of that plan's, so they fit.
int upload_plan(rta_ctx* c, const Plan& plan, PlanDev& d, const std::vector<int32_t>& live,
                hipStream_t s) {
  const size_t mb = (size_t)c->max_items, mt = (size_t)c->max_tier_items;
  std::vector<Item> all_b((size_t)c->n_phase * mb, Item{}), all_t((size_t)c->n_phase * mt, Item{});
  std::vector<int32_t> cnt_b(c->n_phase), cnt_t(c->n_phase);
  for (auto& it : all_b) it.kind = K_NOP;
  for (auto& it : all_t) it.kind = K_NOP;
  int grid = 0;
  for (int ph = 0; ph < c->n_phase; ++ph) {
    std::vector<Item> lst = plan.block[ph];
    if (lst.size() > mb) {
      lst.erase(std::remove_if(lst.begin(), lst.end(), [](const Item& it) { return it.kind == K_NOP; }),
                lst.end());
      if (lst.size() > mb) return RTA_E_STATE;
    }
    if (plan.tier[ph].size() > mt) return RTA_E_STATE;
    std::copy(lst.begin(), lst.end(), all_b.begin() + (size_t)ph * mb);
    std::copy(plan.tier[ph].begin(), plan.tier[ph].end(), all_t.begin() + (size_t)ph * mt);
    cnt_b[ph] = (int32_t)lst.size();
    cnt_t[ph] = (int32_t)plan.tier[ph].size();
    grid = std::max(grid, cnt_b[ph]);
  }
  HIP_TRY(c, hipMemcpyAsync(d.items, all_b.data(), sizeof(Item) * all_b.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(d.phase_count, cnt_b.data(), sizeof(int32_t) * cnt_b.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(d.tier_items, all_t.data(), sizeof(Item) * all_t.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(d.tier_count, cnt_t.data(), sizeof(int32_t) * cnt_t.size(), hipMemcpyHostToDevice, s));
  for (int t = 0; t < c->n_tiers; ++t) {
    const TierHost& T = c->tier[t];
    HIP_TRY(c, hipMemcpyAsync(d.pair_row[t], T.row.data(), sizeof(int64_t) * T.row.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(d.pair_K[t], T.kp.data(), sizeof(int32_t) * T.kp.size(), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(c, hipMemcpyAsync(d.live, live.data(), sizeof(int32_t) * live.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  d.tier_count_host = cnt_t;
  d.block_count_host = cnt_b;
  d.grid_items = grid;
  return RTA_OK;
}

// Work lists of a new serving context: buffers sized by the plan with every
// slot present at max_taps, and the empty plan in buffer 0.
int serve_lists(rta_ctx* c, Plan& plan) {
  Serve* sv = c->serve;
  int st;
  for (int t = 0; t < c->n_tiers; ++t) std::fill(c->tier[t].kp.begin(), c->tier[t].kp.end(), c->tier[t].kcap);
  Plan cap;
  if ((st = build_plan(c, cap)) != RTA_OK) return st;
  for (int t = 0; t < c->n_tiers; ++t) std::fill(c->tier[t].kp.begin(), c->tier[t].kp.end(), 0);
  if ((st = build_plan(c, plan)) != RTA_OK) return st;
  // the slot layout must not depend on which sources are present
  if (cap.tier_slot0 != plan.tier_slot0 || cap.tier_nslot != plan.tier_nslot ||
      cap.groups.size() != plan.groups.size())
    return RTA_E_STATE;
  for (size_t g = 0; g < cap.groups.size(); ++g)
    if (cap.groups[g].slot0 != plan.groups[g].slot0 || cap.groups[g].nslot != plan.groups[g].nslot)
      return RTA_E_STATE;
  c->n_groups = (int)plan.groups.size();
  c->head_slots = (c->L + kXcds - 1) / kXcds * kXcds;
  size_t mb = 1, mt = 1;
  for (int ph = 0; ph < c->n_phase; ++ph) {
    mb = std::max(mb, cap.block[ph].size());
    mt = std::max(mt, cap.tier[ph].size());
  }
  c->max_items = (int)mb;
  c->max_tier_items = (int)mt;
  for (PlanDev& d : sv->dev) {
    if ((st = dev_alloc(c, &d.items, (size_t)c->n_phase * mb)) != RTA_OK) return st;
    if ((st = dev_alloc(c, &d.phase_count, (size_t)c->n_phase)) != RTA_OK) return st;
    if ((st = dev_alloc(c, &d.tier_items, (size_t)c->n_phase * mt)) != RTA_OK) return st;
    if ((st = dev_alloc(c, &d.tier_count, (size_t)c->n_phase)) != RTA_OK) return st;
    for (int t = 0; t < c->n_tiers; ++t) {
      if ((st = dev_alloc(c, &d.pair_row[t], c->tier[t].row.size())) != RTA_OK) return st;
      if ((st = dev_alloc(c, &d.pair_K[t], c->tier[t].kp.size())) != RTA_OK) return st;
    }
    if ((st = dev_alloc(c, &d.live, (size_t)c->Q)) != RTA_OK) return st;
  }
  const std::vector<int32_t> live((size_t)c->Q, 0);
  if ((st = upload_plan(c, plan, sv->dev[0], live, c->stream)) != RTA_OK) return st;
  sv->active = 0;
  activate(c, sv->dev[0]);
  // admissions: staging for one source's taps and spectrum rows
  sv->stage_floats = std::max<int64_t>(sv->cfg.max_taps, kStageBytes / 4);
  sv->row_cap = sv->stage_floats / c->tier[0].span + c->L + 1;
  if ((st = dev_alloc(c, &sv->d_stage, (size_t)sv->stage_floats)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &sv->d_rows, (size_t)sv->row_cap)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &sv->d_range, 1)) != RTA_OK) return st;
  HIP_TRY(c, hipStreamCreateWithFlags(&sv->aux, hipStreamNonBlocking));
  for (hipEvent_t& e : sv->retire) HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return RTA_OK;
}

int create_impl(rta_ctx* c, const std::vector<int>& size, const std::vector<int>& count,
                const float* const* filters, const int64_t* lengths) {
  int st;
  HIP_TRY(c, hipGetDevice(&c->device));
  HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));

  // serving: the arena holds `scale` of the spectra of every slot at
  // max_taps on every output (the lengths passed here), at least one filter
  // per tier
  Serve* sv = c->serve;
  const size_t eb = spectra_elem_bytes(c->dtype);
  double scale = 1.0;
  if (sv != nullptr && sv->cfg.arena_bytes > 0) {
    double full = 0;
    int64_t o = 0;
    for (size_t t = 0; t < size.size(); ++t) {
      const int64_t kc = std::min<int64_t>(count[t] > 0 ? count[t] : INT32_MAX,
                                           std::max<int64_t>(0, (sv->cfg.max_taps - o + size[t] - 1) / size[t]));
      full += (double)c->Q * c->L * kc * size[t] * eb;
      o += (count[t] > 0 ? count[t] : kc) * (int64_t)size[t];
    }
    scale = std::min(1.0, (double)sv->cfg.arena_bytes / std::max(1.0, full));
  }

  // tiers and partition counts
  c->n_tiers = (int)size.size();
  int64_t off = 0;
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    T.P = size[t];
    T.logP = ilog2(T.P);
    T.span = T.P;
    if (c->flags & RTA_FLAG_NF3) {  // validated: one tier, size B
      T.r3 = 1;
      T.P = 3 * c->B / 2;
      T.logP = ilog2(c->B / 2);
    }
    T.offset = off;
    T.row.assign((size_t)c->Q * c->L, -1);
    T.kp.assign((size_t)c->Q * c->L, 0);
    int64_t rows = 0;
    int kmax = 0;
    for (int l = 0; l < c->L; ++l)
      for (int q = 0; q < c->Q; ++q) {
        const int64_t len = lengths[q * c->L + l];
        int64_t need = len > off ? (len - off + T.span - 1) / T.span : 0;
        if (count[t] > 0) need = std::min<int64_t>(need, count[t]);
        const int pair = l * c->Q + q;
        kmax = std::max<int>(kmax, (int)need);
        if (sv != nullptr) continue;  // no source yet
        T.kp[pair] = (int)need;
        if (need > 0) {
          T.row[pair] = rows;
          rows += need;
        }
      }
    T.count = count[t] > 0 ? count[t] : kmax;
    T.K = std::max(t == 0 ? c->min_ring : 1, kmax);
    off += (int64_t)T.count * T.span;
    if (sv != nullptr) {
      T.kcap = kmax;
      const int64_t full = (int64_t)c->Q * c->L * kmax;
      rows = std::max<int64_t>(kmax, (int64_t)std::floor(scale * (double)full));
      rows = std::min(rows, full);
      sv->arena[t].reset(rows);
    }
    const double per_block = (double)c->B / T.span;  // a tier's frame recurs every P/B blocks
    c->spectra_bytes += rows * T.P * (int64_t)eb;
    c->h_bytes += (double)rows * T.P * eb * per_block;
    c->cmacs += (double)rows * T.P * per_block;
    c->x_bytes += (double)c->Q * kmax * T.P * 8.0 * per_block;
    if (t == 0) {
      double tail_rows = 0;
      for (int32_t kp : T.kp) tail_rows += std::max(0, kp - 2);
      c->tail_bytes = tail_rows * T.P * eb + (double)c->Q * std::max(0, kmax - 2) * T.P * 8.0;
    }
    T.h_rows = std::max<int64_t>(1, rows);
    if ((st = dev_alloc(c, reinterpret_cast<char**>(&T.H), (size_t)T.h_rows * T.P * eb)) != RTA_OK)
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
  if (sv != nullptr) c->h_bytes = c->x_bytes = c->cmacs = c->tail_bytes = 0;  // per list
  c->io_bytes = 4.0 * c->B * (c->Q + c->L);
  c->hist_len = std::max<int64_t>(2 * c->B, 2 * (int64_t)c->tier[c->n_tiers - 1].P);
  c->hist_len = int64_t(1) << ilog2(c->hist_len);
  // later tiers store each frame's output up to o_t samples ahead of the
  // block being emitted (their time-domain delay)
  c->ring_len = 1;
  if (c->n_tiers > 1) c->ring_len = int64_t(1) << ilog2(c->tier[c->n_tiers - 1].offset + 2 * c->B);
  for (int t = 1; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    if ((st = dev_alloc(c, &T.oring, (size_t)c->L * c->ring_len)) != RTA_OK) return st;
    if ((st = dev_alloc(c, &T.tfwd, (size_t)c->Q * T.P)) != RTA_OK) return st;
    if ((st = dev_alloc(c, &T.tinv, (size_t)c->L * T.P)) != RTA_OK) return st;
  }

  // spectra, then the heads' dense copy of partitions 0 and 1 (serving: no
  // source yet, so the copy starts as zeros)
  if (sv == nullptr && (st = build_spectra(c, filters, lengths)) != RTA_OK) return st;
  if ((st = dev_alloc(c, reinterpret_cast<char**>(&c->H01), (size_t)c->L * c->Q * 2 * c->tier[0].P * eb)) != RTA_OK)
    return st;
  HIP_TRY(c, launch_gather(c->dtype, c->tier[0], c->L * c->Q, c->H01, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  // outputs per group: as requested, halved until a head's LDS fits
  int max_lds = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));


  // work lists
  Plan plan;
  if (sv != nullptr) {
    if ((st = serve_lists(c, plan)) != RTA_OK) return st;
  } else {
  if ((st = build_plan(c, plan)) != RTA_OK) return st;
  c->n_groups = (int)plan.groups.size();
  c->head_slots = (c->L + kXcds - 1) / kXcds * kXcds;  // keeps tails' XCD residues
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
  c->block_count_host = cnt_b;
  if ((st = dev_alloc(c, &c->items, all_b.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->phase_count, cnt_b.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_items, all_t.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_count, cnt_t.size())) != RTA_OK) return st;
  HIP_TRY(c, hipMemcpy(c->items, all_b.data(), sizeof(Item) * all_b.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->phase_count, cnt_b.data(), sizeof(int32_t) * cnt_b.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->tier_items, all_t.data(), sizeof(Item) * all_t.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->tier_count, cnt_t.data(), sizeof(int32_t) * cnt_t.size(), hipMemcpyHostToDevice));
  c->grid_items = c->max_items;
  }
  if ((st = dev_alloc(c, &c->tier_slot0, plan.tier_slot0.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->tier_nslot, plan.tier_nslot.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->groups, plan.groups.size())) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->head_count, 1)) != RTA_OK) return st;
  if ((st = dev_alloc(c, &c->heads_done, 1)) != RTA_OK) return st;
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
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_status), sizeof(int32_t),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return RTA_E_NOMEM;
  }
  __atomic_store_n(c->h_status, 0, __ATOMIC_RELEASE);
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_in), c->h_in, 0));
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_out), c->h_out, 0));
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_flag), c->h_flag, 0));
  HIP_TRY(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->m_status), c->h_status, 0));

  // LDS: the larger of a head's layout (HeadLds) and a tail item's row-group
  // reduction.  head_nq: as many inputs per pass as fit in 48 KB, at least 1.
  const int C = vec_bins(c->dtype);
  // uniform partitions re-read every spectrum row every block: ordinary
  // loads stream them faster up to a few hundred MB (measured with 61 to
  // 295 MB of spectra, inside and beyond the 256 MB Infinity Cache), while
  // 443 MB (4 -> 64 x U[3,12] s FP16) went faster non-temporal; later tiers
  // touch their rows once per frame, and serving contexts stream whatever
  // is admitted: non-temporal loads there
  c->nt = c->spectra_loads == 1 ||
          (c->spectra_loads == 0 && (c->serve != nullptr || c->n_tiers > 1 ||
                                     c->spectra_bytes > (int64_t(384) << 20)));
  const int P0 = c->tier[0].P;
  const int fixed = head_lds(P0, 1, 1).total - 2 * P0;
  c->head_nq = std::max(1, std::min(c->Q, (6144 - fixed) / (2 * P0)));
  // With later tiers, also a transform pass's buffers (kTierLds).
  c->lds = sizeof(float2) * std::max((size_t)head_lds(P0, 1, c->head_nq).total,
                                     (size_t)kThreads * C * c->G);
  if (c->n_tiers > 1) c->lds = std::max(c->lds, sizeof(float2) * (size_t)kTierLds);
  if ((int64_t)c->lds + 64 > (int64_t)max_lds) return RTA_E_UNSUPPORTED;
  if (c->lds > 65536)
    HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(block_kernel(c->dtype, c->G, c->nt)),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds));
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
  if (c->serve) {
    if (c->serve->aux) {
      (void)hipStreamSynchronize(c->serve->aux);
      (void)hipStreamDestroy(c->serve->aux);
    }
    for (hipEvent_t e : c->serve->retire)
      if (e) (void)hipEventDestroy(e);
    delete c->serve;
    c->serve = nullptr;
  }
  for (void* p : c->dev_allocs) (void)hipFree(p);
  c->dev_allocs.clear();
  c->n_dev = nullptr;
  c->n_dev_value = -1;
  if (c->h_in) (void)hipHostFree(c->h_in);
  if (c->h_out) (void)hipHostFree(c->h_out);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->h_status) (void)hipHostFree(c->h_status);
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
  // partition ratio between tiers, largest partition, and how many times
  // its minimum length the first (block-sized) tier covers
  for (int ratio : {8, 4})
    for (int64_t cap : {8192, 2048})
      for (int first : {1, 2}) {
        std::vector<std::pair<int, int>> sch;
        int64_t o = 0;
        int64_t P = B;
        while (true) {
          const int64_t Pn = P * ratio;
          // a tier starts at least 2 P - B in (P / B blocks of slack) and at
          // least P + 4 B; counts are whole partitions
          int64_t on = std::max<int64_t>(2 * Pn - B, Pn + 4 * (int64_t)B);
          if (sch.empty()) on *= first;
          const int64_t count = (on - o + P - 1) / P;
          on = o + count * P;
          if (Pn > cap || max_len <= on) break;
          sch.push_back({(int)P, (int)count});
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

// ---------------------------------------------------------------------------
// Serving: control calls (hold sv->ctl).
// ---------------------------------------------------------------------------

bool present(int state) { return state != RTA_SLOT_FREE; }

// Return the arena rows of slots that have become free.
void reclaim(Serve* sv, int n_tiers) {
  std::vector<int> freed;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (size_t q = 0; q < sv->slots.size(); ++q)
      if (sv->slots[q].state == RTA_SLOT_FREE && sv->slots[q].rows_held) freed.push_back((int)q);
  }
  for (int q : freed) {
    ServeSlot& sl = sv->slots[q];
    for (int t = 0; t < n_tiers; ++t) {
      for (size_t l = 0; l < sl.row[t].size(); ++l)
        if (sl.row[t][l] >= 0) sv->arena[t].release(sl.row[t][l], sl.kp[t][l]);
      sl.row[t].clear();
      sl.kp[t].clear();
    }
    sl.rows_held = false;
  }
}

// Build the work list for the slot states `states` (one slot may be given a
// state it will take when the list is published), write it into the
// buffer launches are not reading, and publish it: the next block switches
// to it.  `after` is applied to the slot states in the same critical section
// that publishes the list.  gather: refresh the heads' copy of partitions 0
// and 1 from the new pair tables first.
template <typename F>
int commit_plan(rta_ctx* c, std::vector<int> states, bool gather, F after) {
  Serve* sv = c->serve;
  const int Q = c->Q, L = c->L;
  int st;
  PlanDev tmp;  // per-block figures of the new list
  for (int t = 0; t < c->n_tiers; ++t) {
    TierHost& T = c->tier[t];
    std::fill(T.row.begin(), T.row.end(), -1);
    std::fill(T.kp.begin(), T.kp.end(), 0);
  }
  std::vector<int32_t> live((size_t)Q, 0);
  for (int q = 0; q < Q; ++q) {
    if (!present(states[q])) continue;
    const ServeSlot& sl = sv->slots[q];
    live[q] = (states[q] == RTA_SLOT_JOINING || states[q] == RTA_SLOT_LIVE) ? 1 : 0;
    for (int t = 0; t < c->n_tiers; ++t)
      for (int l = 0; l < L; ++l) {
        c->tier[t].row[(size_t)l * Q + q] = sl.row[t][l];
        c->tier[t].kp[(size_t)l * Q + q] = sl.kp[t][l];
      }
    tmp.hb += sl.hb;
    tmp.xb += sl.xb;
    tmp.cm += sl.cm;
  }
  {
    const TierHost& T = c->tier[0];
    const size_t ebytes = spectra_elem_bytes(c->dtype);
    double tail_rows = 0;
    std::vector<int> kq((size_t)Q, 0);
    for (int l = 0; l < L; ++l)
      for (int q = 0; q < Q; ++q) {
        const int kp = T.kp[(size_t)l * Q + q];
        tail_rows += std::max(0, kp - 2);
        kq[q] = std::max(kq[q], kp);
      }
    double xr = 0;
    for (int k : kq) xr += std::max(0, k - 2);
    tmp.tb = tail_rows * T.P * ebytes + xr * T.P * 8.0;
  }
  Plan plan;
  if ((st = build_plan(c, plan)) != RTA_OK) return st;

  int target;
  bool wait = false;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    target = sv->active ^ 1;
    if (sv->pending)
      sv->pending = false;  // the other buffer was published but not yet read
    else
      wait = sv->retire_valid[target];
  }
  if (wait) HIP_TRY(c, hipEventSynchronize(sv->retire[target]));
  PlanDev& d = sv->dev[target];
  if ((st = upload_plan(c, plan, d, live, sv->aux)) != RTA_OK) return st;
  if (gather) {
    TierHost T0 = c->tier[0];
    T0.pair_row = d.pair_row[0];
    T0.pair_K = d.pair_K[0];
    HIP_TRY(c, launch_gather(c->dtype, T0, L * Q, c->H01, sv->aux));
    HIP_TRY(c, hipStreamSynchronize(sv->aux));
  }
  d.hb = tmp.hb;
  d.xb = tmp.xb;
  d.cm = tmp.cm;
  d.tb = tmp.tb;
  std::lock_guard<std::mutex> lk(sv->mu);
  after();
  sv->pending = true;
  return RTA_OK;
}

std::vector<int> slot_states(Serve* sv) {
  std::lock_guard<std::mutex> lk(sv->mu);
  std::vector<int> st;
  for (const ServeSlot& sl : sv->slots) st.push_back(sl.state);
  return st;
}

// noalloc: stage the spectra build in this device's scratch array instead of
// the context's staging buffers.
int serve_admit(rta_ctx* c, const float* const* filters, const int64_t* lengths, int32_t* slot,
                bool noalloc) {
  Serve* sv = c->serve;
  const int L = c->L;
  std::lock_guard<std::mutex> cl(sv->ctl);
  if (c->poisoned) return RTA_E_DEVICE;
  reclaim(sv, c->n_tiers);

  // partitions per tier of each of the source's filters, and what it streams
  const size_t eb = spectra_elem_bytes(c->dtype);
  ServeSlot src;
  for (int l = 0; l < L; ++l) src.taps = std::max(src.taps, lengths[l]);
  for (int t = 0; t < c->n_tiers; ++t) {
    const TierHost& T = c->tier[t];
    const double per_block = (double)c->B / T.P;
    src.row[t].assign((size_t)L, -1);
    src.kp[t].assign((size_t)L, 0);
    int kmax = 0;
    for (int l = 0; l < L; ++l) {
      const int64_t len = lengths[l];
      int64_t need = len > T.offset ? (len - T.offset + T.P - 1) / T.P : 0;
      need = std::min<int64_t>(need, T.count);
      src.kp[t][l] = (int)need;
      kmax = std::max(kmax, (int)need);
      src.hb += (double)need * T.P * eb * per_block;
      src.cm += (double)need * T.P * per_block;
    }
    src.xb += (double)kmax * T.P * 8.0 * per_block;
  }

  int q = -1;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    double bytes = 0;
    for (const ServeSlot& sl : sv->slots)
      if (present(sl.state)) bytes += sl.hb + sl.xb;
    for (size_t i = 0; i < sv->slots.size() && q < 0; ++i)
      if (sv->slots[i].state == RTA_SLOT_FREE && !sv->slots[i].rows_held) q = (int)i;
    if (q < 0) {
      ++sv->rej_slots;
      return RTA_E_CAPACITY;
    }
    if (sv->cfg.budget_bytes > 0 && bytes + src.hb + src.xb > sv->cfg.budget_bytes) {
      ++sv->rej_budget;
      return RTA_E_CAPACITY;
    }
  }

  // arena rows: one contiguous range per (tier, output)
  auto give_back = [&]() {
    for (int t = 0; t < c->n_tiers; ++t)
      for (int l = 0; l < L; ++l)
        if (src.row[t][l] >= 0) {
          sv->arena[t].release(src.row[t][l], src.kp[t][l]);
          src.row[t][l] = -1;
        }
  };
  for (int t = 0; t < c->n_tiers; ++t)
    for (int l = 0; l < L; ++l) {
      if (src.kp[t][l] == 0) continue;
      src.row[t][l] = sv->arena[t].alloc(src.kp[t][l]);
      if (src.row[t][l] < 0) {
        give_back();
        std::lock_guard<std::mutex> lk(sv->mu);
        ++sv->rej_mem;
        return RTA_E_NOMEM;
      }
    }

  // spectra into those rows (no launch reads them yet)
  std::vector<SpecJob> jobs;
  for (int t = 0; t < c->n_tiers; ++t)
    for (int l = 0; l < L; ++l)
      if (src.kp[t][l] > 0) jobs.push_back(SpecJob{t, filters[l], lengths[l], src.row[t][l], src.kp[t][l]});
  int st;
  if (noalloc) {
    unsigned char* base = static_cast<unsigned char*>(scratch_on(c->device));
    if (base == nullptr) {
      st = RTA_E_DEVICE;
    } else {
      std::lock_guard<std::mutex> use(g_scratch_use[c->device]);
      st = run_spectra(c, jobs, sv->aux, reinterpret_cast<float*>(base + kScratchTapsOff), kScratchTaps,
                       reinterpret_cast<SpecRow*>(base + kScratchRowsOff), kScratchRows,
                       reinterpret_cast<int*>(base));
    }
  } else {
    st = run_spectra(c, jobs, sv->aux, sv->d_stage, sv->stage_floats, sv->d_rows, sv->row_cap,
                     sv->d_range);
  }
  if (st != RTA_OK) {
    give_back();
    return st;
  }

  ServeSlot& sl = sv->slots[q];  // FREE and without rows: only this call touches it
  for (int t = 0; t < c->n_tiers; ++t) {
    sl.row[t] = src.row[t];
    sl.kp[t] = src.kp[t];
  }
  sl.taps = src.taps;
  sl.hb = src.hb;
  sl.xb = src.xb;
  sl.cm = src.cm;
  sl.rows_held = true;
  sl.start = sl.stop = sl.free_at = -1;
  std::vector<int> states = slot_states(sv);
  states[q] = RTA_SLOT_JOINING;
  st = commit_plan(c, states, true, [&]() {
    sv->slots[q].state = RTA_SLOT_JOINING;
    ++sv->admitted;
  });
  if (st != RTA_OK) {
    give_back();
    for (int t = 0; t < c->n_tiers; ++t) {
      sl.row[t].clear();
      sl.kp[t].clear();
    }
    sl.rows_held = false;
    return st;
  }
  *slot = q;
  return RTA_OK;
}

int serve_release(rta_ctx* c, int32_t q) {
  Serve* sv = c->serve;
  std::lock_guard<std::mutex> cl(sv->ctl);
  if (c->poisoned) return RTA_E_DEVICE;
  std::vector<int> states = slot_states(sv);
  if (states[q] != RTA_SLOT_JOINING && states[q] != RTA_SLOT_LIVE) return RTA_E_STATE;
  states[q] = RTA_SLOT_LEAVING;
  return commit_plan(c, states, false, [&]() { sv->slots[q].state = RTA_SLOT_LEAVING; });
}

// rta_reset for a serving context: the device is idle; zero the state, keep
// the live sources (live from block 0) and free the released ones.
int serve_reset(rta_ctx* c) {
  Serve* sv = c->serve;
  std::lock_guard<std::mutex> cl(sv->ctl);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (ServeSlot& sl : sv->slots) {
      if (sl.state == RTA_SLOT_JOINING || sl.state == RTA_SLOT_LIVE) {
        sl.state = RTA_SLOT_LIVE;
        sl.start = 0;
        sl.stop = sl.free_at = -1;
      } else if (sl.state != RTA_SLOT_FREE) {
        sl.state = RTA_SLOT_FREE;
      }
    }
  }
  reclaim(sv, c->n_tiers);
  // publish a list without the freed slots, then switch to it right away
  int st = commit_plan(c, slot_states(sv), true, []() {});
  if (st != RTA_OK) return st;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->active ^= 1;
    sv->pending = false;
    sv->retire_valid[0] = sv->retire_valid[1] = false;
    activate(c, sv->dev[sv->active]);
  }
  return zero_state(c);
}

bool tuning_ok(const rta_tuning* tuning) {
  if (tuning == nullptr) return true;
  const int g = tuning->outputs_per_group;
  const int s = tuning->bin_slices;
  return !((g != 0 && g != 1 && g != 2 && g != 4) || tuning->tail_items < 0 || tuning->tail_rows < 0 ||
           tuning->tier_rows < 0 || (s != 0 && s != 1 && s != 2 && s != 4 && s != 8) ||
           tuning->spectra_loads < 0 || tuning->spectra_loads > 2);
}

int create_ctx(rta_ctx** out, double fs, int32_t block, const std::vector<int>& size,
               const std::vector<int>& count, int32_t n_in, int32_t n_out,
               const float* const* filters, const int64_t* lengths, int32_t spectra,
               uint32_t flags, const rta_tuning* tuning, const rta_serve_config* cfg,
               int min_ring = 1) {
  rta_ctx* c = new (std::nothrow) rta_ctx();
  if (c == nullptr) return RTA_E_NOMEM;
  c->min_ring = min_ring;
  c->fs = fs;
  c->B = block;
  c->Q = n_in;
  c->L = n_out;
  c->dtype = spectra;
  c->flags = flags;
  // tiling defaults from sweeps on MI355X (1 -> 32 x 480,000 taps, 1 -> 64 x
  // 576,000 taps, FP32 and FP16, uniform; 4 -> 64 x U[3,12] s, FP16,
  // 128/1024/8192): about 512 first-tier items, two outputs per workgroup
  // from 16 outputs on, four with later tiers and 64 outputs or more
  c->G = (size.size() > 1 && n_out >= 64) ? 4 : n_out >= 16 ? 2 : 1;
  // 16-bit spectra larger than half the 256 MB Infinity Cache stream mostly
  // from HBM even in a context of their own; there the delay-line reads
  // (FP32, through the vector caches) weigh more than the halved spectrum
  // bytes, and four outputs per read with two bin slices pay (measured with
  // the cache defeated, 1 -> 64 x 576,000 taps FP16: 33.1 -> 31.0 us per
  // block; in one context unchanged)
  bool big16 = false, uni16 = false;
  if (size.size() == 1 && spectra != RTA_FP32 && cfg == nullptr && !(flags & RTA_FLAG_NF3) && n_out >= 32) {
    uni16 = true;
    double rows = 0;
    for (int64_t i = 0; i < (int64_t)n_in * n_out; ++i) rows += (double)((lengths[i] + block - 1) / block);
    big16 = rows * block * 4.0 > 128.0 * (1 << 20);
    if (big16) c->G = 4;
  }
  if (tuning != nullptr) {
    if (tuning->outputs_per_group) c->G = tuning->outputs_per_group;
    if (tuning->tail_items) c->tail_items = tuning->tail_items;
    if (tuning->tail_rows) c->rows_per_item = tuning->tail_rows;
    if (tuning->tier_rows) c->tier_rows = tuning->tier_rows;
    if (tuning->bin_slices) c->bin_slices = tuning->bin_slices;
    c->spectra_loads = tuning->spectra_loads;
  }
  // 16-bit spectra under uniform partitions: two bin slices unless the
  // caller chose (1 -> 32 x 10 s: 14.07 -> 13.93 us per block, and 0.452 ->
  // 0.461 of HBM peak with the cache defeated)
  if (uni16 && c->bin_slices == 0) c->bin_slices = 2;
  if (cfg != nullptr) {
    c->serve = new (std::nothrow) Serve();
    if (c->serve == nullptr) {
      delete c;
      return RTA_E_NOMEM;
    }
    c->serve->cfg = *cfg;
    c->serve->slots.resize((size_t)n_in);
  }
  const int st = create_impl(c, size, count, filters, lengths);
  if (st != RTA_OK) {
    free_all(c);
    delete c;
    return st;
  }
  *out = c;
  return RTA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Tuning cache: one JSON object per line, keyed by everything the autotuner's
// choice depends on (device, rate, block, shape, filter lengths, spectra
// type, flags, scheme or "auto", trial length); filter values do not enter.
// ---------------------------------------------------------------------------
std::string tuning_key(double fs, int32_t block, const rta_scheme* scheme, int32_t n_in,
                       int32_t n_out, const int64_t* lengths, int32_t spectra, uint32_t flags,
                       int32_t blocks) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  (void)hipGetLastError();
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the lengths
  for (int64_t i = 0; i < (int64_t)n_in * n_out; ++i) {
    uint64_t v = (uint64_t)lengths[i];
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  }
  // "auto" names the candidate set of scheme_candidates(): a changed set
  // gets a new name so that older entries miss
  std::string sch = "auto2";
  if (scheme != nullptr) {
    sch.clear();
    for (int t = 0; t < scheme->n_tiers; ++t)
      sch += (t ? "," : "") + std::to_string(scheme->size[t]) + "x" + std::to_string(scheme->count[t]);
  }
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s;cu=%d;fs=%.17g;B=%d;Q=%d;L=%d;len=%016llx;spectra=%d;flags=%u;blocks=%d;scheme=%s",
                arch.c_str(), cus, fs, block, n_in, n_out, (unsigned long long)h, spectra, flags,
                blocks, sch.c_str());
  // the key sits inside a JSON string: keep it free of quotes and backslashes
  std::string k = buf;
  for (char& ch : k)
    if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20) ch = '_';
  return k;
}

// Parse the integers of `"name": [a, b, ...]` or `"name": a` after `from`.
bool json_ints(const std::string& line, const char* name, int32_t* v, int n) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  const char* p = line.c_str() + at + pat.size();
  while (*p == ' ') ++p;
  const bool arr = *p == '[';
  if (arr) ++p;
  for (int i = 0; i < n; ++i) {
    char* end = nullptr;
    const long x = std::strtol(p, &end, 10);
    if (end == p) return false;
    v[i] = (int32_t)x;
    p = end;
    while (*p == ' ' || *p == ',') ++p;
  }
  return !arr || *p == ']';
}

bool cache_lookup(const char* path, const std::string& key, rta_tuning* t, double* us) {
  FILE* fp = std::fopen(path, "r");
  if (fp == nullptr) return false;
  const std::string want = "{\"key\": \"" + key + "\",";
  std::string line;
  bool found = false;
  char chunk[1024];
  while (std::fgets(chunk, sizeof chunk, fp) != nullptr) {
    line += chunk;
    if (line.empty() || line.back() != '\n') continue;  // a longer line: keep reading
    if (line.compare(0, want.size(), want) == 0) {
      rta_tuning c{};
      bool ok = json_ints(line, "outputs_per_group", &c.outputs_per_group, 1) &&
                json_ints(line, "tail_items", &c.tail_items, 1) &&
                json_ints(line, "tail_rows", &c.tail_rows, 1) &&
                json_ints(line, "tier_rows", &c.tier_rows, 1) &&
                json_ints(line, "bin_slices", &c.bin_slices, 1) &&
                json_ints(line, "n_tiers", &c.n_tiers, 1);
      ok = ok && c.n_tiers >= 1 && c.n_tiers <= RTA_MAX_TIERS &&
           json_ints(line, "size", c.size, c.n_tiers) && json_ints(line, "count", c.count, c.n_tiers);
      if (!json_ints(line, "spectra_loads", &c.spectra_loads, 1)) c.spectra_loads = 0;  // optional
      const size_t at = line.find("\"us\":");
      if (ok && at != std::string::npos) {
        *t = c;  // the last matching line wins
        *us = std::strtod(line.c_str() + at + 5, nullptr);
        found = true;
      }
    }
    line.clear();
  }
  std::fclose(fp);
  return found;
}

int cache_append(const char* path, const std::string& key, const rta_tuning& t, double us) {
  std::string line = "{\"key\": \"" + key + "\", \"outputs_per_group\": " +
                     std::to_string(t.outputs_per_group) + ", \"tail_items\": " +
                     std::to_string(t.tail_items) + ", \"tail_rows\": " + std::to_string(t.tail_rows) +
                     ", \"tier_rows\": " + std::to_string(t.tier_rows) + ", \"bin_slices\": " +
                     std::to_string(t.bin_slices) + ", \"spectra_loads\": " +
                     std::to_string(t.spectra_loads) + ", \"n_tiers\": " + std::to_string(t.n_tiers);
  std::string sz, ct;
  for (int i = 0; i < t.n_tiers; ++i) {
    sz += (i ? ", " : "") + std::to_string(t.size[i]);
    ct += (i ? ", " : "") + std::to_string(t.count[i]);
  }
  char usb[64];
  std::snprintf(usb, sizeof usb, "%.3f", us);
  line += ", \"size\": [" + sz + "], \"count\": [" + ct + "], \"us\": " + usb + "}\n";
  FILE* fp = std::fopen(path, "a");
  if (fp == nullptr) return RTA_E_ARG;
  const bool ok = std::fputs(line.c_str(), fp) >= 0;
  return (std::fclose(fp) == 0 && ok) ? RTA_OK : RTA_E_ARG;
}

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
  if (!tuning_ok(tuning)) return RTA_E_ARG;
  return create_ctx(out, fs, block, size, count, n_in, n_out, filters, lengths, spectra, flags,
                    tuning, nullptr);
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
  using clk = std::chrono::steady_clock;
  const clk::time_point ta = clk::now();
  std::memcpy(c->h_in, in, sizeof(float) * (size_t)c->Q * c->B);
  const int64_t want = c->block + 1;
  const clk::time_point tb = clk::now();
  int st = launch_block(c, c->m_in, c->m_out, c->stream, true);
  if (st != RTA_OK) return st;
  // spin until the last head has raised the flag; the tail workgroups of the
  // same launch keep running.  No runtime call on the normal path: only once
  // the flag is 2 ms late is the stream asked for errors (then every 1 ms),
  // so a failed launch cannot spin forever.
  const clk::time_point t0 = clk::now();
  clk::time_point next_check = t0 + std::chrono::milliseconds(2);
  for (uint64_t i = 1;; ++i) {
    if (__atomic_load_n(c->h_flag, __ATOMIC_ACQUIRE) == want) break;
    if ((i & 255) == 0 && clk::now() >= next_check) {
      if (next_check == t0 + std::chrono::milliseconds(2)) c->hs.late += 1;
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipSuccess) {
        if (__atomic_load_n(c->h_flag, __ATOMIC_ACQUIRE) == want) break;
        c->poisoned = true;
        return RTA_E_DEVICE;
      }
      if (e != hipErrorNotReady) HIP_TRY(c, e);
      next_check = clk::now() + std::chrono::milliseconds(1);
    }
  }
  if ((st = device_status(c)) != RTA_OK) return st;
  const clk::time_point td = clk::now();
  std::memcpy(out, c->h_out, sizeof(float) * (size_t)c->L * c->B);
  const clk::time_point te = clk::now();
  const clk::time_point ts[5] = {ta, tb, t0, td, te};
  rta_ctx::HostStages& h = c->hs;
  for (int k = 0; k < 4; ++k) {
    const double us = std::chrono::duration<double, std::micro>(ts[k + 1] - ts[k]).count();
    h.max_us[k] = std::max(h.max_us[k], us);
    h.sum_us[k] += us;
  }
  const double tot = std::chrono::duration<double, std::micro>(te - ta).count();
  if (tot > h.slowest_us) {
    h.slowest_us = tot;
    h.slowest_call = h.calls;
  }
  h.calls += 1;
  return RTA_OK;
}

int rta_process_device(rta_ctx* c, const float* d_in, float* d_out, void* stream) {
  if (c == nullptr || d_in == nullptr || d_out == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  const int st = device_status(c);  // set by a block launched earlier
  if (st != RTA_OK) return st;
  return launch_block(c, d_in, d_out, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Graph replay: n consecutive block launches captured once into a hipGraph.
// Each captured launch carries its place j in the run; the kernels take the
// block index as *n_dev + j, and the graph's last node advances n_dev by n,
// so every replay processes the next n blocks without re-capture or
// per-launch arguments from the host.
// ---------------------------------------------------------------------------
struct rta_graph {
  rta_ctx* c = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t n_blocks = 0;
  int64_t block0 = 0;      // context block index at capture
  int64_t config_gen = 0;
};

int rta_graph_create(rta_ctx* c, const float* d_in, float* d_out, int32_t n_blocks,
                     rta_graph** out) {
  if (out == nullptr) return RTA_E_ARG;
  *out = nullptr;
  if (c == nullptr || d_in == nullptr || d_out == nullptr || n_blocks < 1) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  if (c->serve != nullptr || (c->fc != nullptr && !c->fc_fused)) return RTA_E_UNSUPPORTED;
  if (n_blocks % c->n_phase != 0) return RTA_E_ARG;
  int st = device_status(c);
  if (st != RTA_OK) return st;
  if (c->n_dev == nullptr && (st = dev_alloc(c, &c->n_dev, 1)) != RTA_OK) return st;
  hipStream_t cs = nullptr;
  HIP_TRY(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int32_t j = 0; j < n_blocks && e == hipSuccess; ++j) {
      KArgs a = make_args(c, d_in + (int64_t)j * c->Q * c->B, d_out + (int64_t)j * c->L * c->B, j);
      a.n_base = c->n_dev;
      unsigned grid = 0;
      size_t lds = 0;
      block_geometry(c, c->block + j, a, grid, lds);
      hipLaunchKernelGGL(block_kernel(c->dtype, c->G, c->nt), dim3(grid), dim3(kThreads), lds, cs, a);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, cs, c->n_dev, (int64_t)n_blocks, 1);
      e = hipGetLastError();
    }
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return RTA_E_DEVICE;  // capture failed; the context itself is untouched
  }
  rta_graph* g = new rta_graph;
  g->c = c;
  g->graph = graph;
  g->exec = exec;
  g->n_blocks = n_blocks;
  g->block0 = c->block;
  g->config_gen = c->config_gen;
  *out = g;
  return RTA_OK;
}

int rta_graph_launch(rta_graph* g, void* stream) {
  if (g == nullptr) return RTA_E_ARG;
  rta_ctx* c = g->c;
  if (c->poisoned) return RTA_E_DEVICE;
  int st = device_status(c);
  if (st != RTA_OK) return st;
  if (g->config_gen != c->config_gen) return RTA_E_STATE;
  if ((c->block - g->block0) % c->n_phase != 0) return RTA_E_STATE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->n_dev_value != c->block) {  // other launches moved the block index
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, c->n_dev, c->block, 0);
    HIP_TRY(c, hipGetLastError());
  }
  HIP_TRY(c, hipGraphLaunch(g->exec, s));
  c->block += g->n_blocks;
  if (c->fc != nullptr) c->fc->block += g->n_blocks;  // fused: ran inside these launches
  c->n_dev_value = c->block;
  return RTA_OK;
}

int rta_graph_destroy(rta_graph* g) {
  if (g == nullptr) return RTA_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return RTA_OK;
}

int rta_reset(rta_ctx* c) {
  if (c == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  HIP_TRY(c, hipDeviceSynchronize());
  const int st = device_status(c);
  if (st != RTA_OK) return st;
  if (c->serve != nullptr) return serve_reset(c);
  return zero_state(c);
}

int rta_query(rta_ctx* c, rta_info* info) {
  if (c == nullptr || info == nullptr) return RTA_E_ARG;
  (void)device_status(c);
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
  info->grid = c->head_slots + c->grid_items;
  info->outputs_per_group = c->G;
  info->rows_per_item = c->rows_per_item;
  info->poisoned = c->poisoned ? 1 : 0;
  info->feedback_paths = c->fc != nullptr ? 1 : 0;
  info->feedback_fused = c->fc != nullptr && c->fc_fused ? 1 : 0;
  info->spectra_nontemporal = c->nt ? 1 : 0;
  info->fft_size = 2 * c->tier[0].P;
  info->host_calls = c->hs.calls;
  for (int k = 0; k < 4; ++k) {
    info->host_max_us[k] = c->hs.max_us[k];
    info->host_sum_us[k] = c->hs.sum_us[k];
  }
  info->host_slowest_call = c->hs.slowest_call;
  info->host_slowest_us = c->hs.slowest_us;
  info->host_late_waits = c->hs.late;
  info->bin_slices = std::max(1, c->bin_slices);
  info->max_group_slots = c->max_group_slots;
  return c->poisoned ? RTA_E_DEVICE : RTA_OK;
}

int rta_set_feedback(rta_ctx* c, const float* const* fb, const int64_t* lengths, int32_t spectra) {
  if (c == nullptr) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  // the feedback convolution runs outputs -> inputs: its filter [l][q] is
  // f_ql; validated like rta_create's arguments (uniform partitions, P = B)
  // before anything is touched
  const int64_t np = (int64_t)c->Q * c->L;
  std::vector<const float*> ft;
  std::vector<int64_t> lt;
  std::vector<int> size, count;
  if (fb != nullptr) {
    if (lengths == nullptr) return RTA_E_ARG;
    ft.resize(np);
    lt.resize(np);
    for (int q = 0; q < c->Q; ++q)
      for (int l = 0; l < c->L; ++l) {
        ft[(int64_t)l * c->Q + q] = fb[(int64_t)q * c->L + l];
        lt[(int64_t)l * c->Q + q] = lengths[(int64_t)q * c->L + l];
      }
    const int st = validate(c->fs, c->B, nullptr, c->L, c->Q, ft.data(), lt.data(), spectra,
                            c->flags & RTA_FLAG_NF3, size, count);
    if (st != RTA_OK) return st;
    // n_f = 3B hands the synthesis spectra to the feedback filters inside the
    // block launch: same spectrum type required
    if ((c->flags & RTA_FLAG_NF3) && spectra != c->dtype) return RTA_E_UNSUPPORTED;
  }
  HIP_TRY(c, hipDeviceSynchronize());
  c->config_gen += 1;  // graphs captured so far no longer match
  if (c->fc) {
    free_all(c->fc);
    delete c->fc;
    c->fc = nullptr;
  }
  c->fc_fused = false;
  if (fb != nullptr) {
    // same outputs per group as this context, so its items can run in this
    // context's launch; at least 3 delay-line slots (this launch writes slot
    // n while its heads read n-1 and n-2)
    rta_tuning tu{};
    tu.outputs_per_group = c->G;
    // its one head per output reduces all of that output's partial slots on
    // the synthesis heads' critical path: 512 items in 8 bin slices keep them
    // to about 64 while its items stay as small as the synthesis tails'
    tu.tail_items = 512;
    tu.bin_slices = 8;
    rta_ctx* fc = nullptr;
    int st = create_ctx(&fc, c->fs, c->B, size, count, c->L, c->Q, ft.data(), lt.data(), spectra,
                        c->flags & RTA_FLAG_NF3, &tu, nullptr, 3);
    if (st != RTA_OK) return st;
    c->fc = fc;
    if (c->d_y == nullptr) {
      if ((st = dev_alloc(c, &c->d_y, (size_t)c->L * c->B)) != RTA_OK) return st;
      if ((st = dev_alloc(c, &c->d_c, (size_t)c->Q * c->B)) != RTA_OK) return st;
      if ((st = dev_alloc(c, &c->fc_done, 1)) != RTA_OK) return st;
    }
    // fused when both store the same spectrum type and the launch's LDS fits
    const int P = c->tier[0].P, C = vec_bins(c->dtype);
    const size_t fc_head = sizeof(float2) * (size_t)(3 * P + tw_lds_len(P) + red_scratch(P));
    const size_t fc_tail = sizeof(float2) * (size_t)kThreads * C * c->G;
    c->lds_fused = std::max(c->lds, std::max(fc_head, fc_tail));
    int max_lds = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    c->fc_fused = fc->dtype == c->dtype && fc->G == c->G && fc->n_tiers == 1 && fc->tier[0].K >= 3 &&
                  fc->tier[0].P == P && (int64_t)c->lds_fused + 64 <= (int64_t)max_lds;
    if (c->fc_fused && c->lds_fused > 65536)
      HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(block_kernel(c->dtype, c->G, c->nt)),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_fused));
    if ((c->flags & RTA_FLAG_NF3) && !c->fc_fused) {  // the hand-off exists only fused
      free_all(c->fc);
      delete c->fc;
      c->fc = nullptr;
      (void)zero_state(c);
      return RTA_E_UNSUPPORTED;
    }
  }
  // serving: the paths belong to the slots; live sources stay, released ones
  // are freed, as rta_reset does
  if (c->serve != nullptr) return serve_reset(c);
  return zero_state(c);
}

int rta_test_feedback_wait(rta_ctx* c, int32_t max_polls, int32_t never_ready) {
  if (c == nullptr || max_polls < 1 || (never_ready != 0 && never_ready != 1)) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  c->fc_wait_polls = max_polls;
  c->fc_wait_bias = never_ready ? 0x40000000u : 0u;
  return RTA_OK;
}

int rta_timing_enable(rta_ctx* c, int32_t every) {
  if (c == nullptr || every < 0) return RTA_E_ARG;
  if (every > 0) c->timing_span_read = every;  // spans recorded from now on
  c->timing = every;
  c->timing_base = c->block;
  c->span_open = false;
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
    *blocks += std::max(1, c->timing_span_read);
  }
  c->events_used = 0;
  c->span_open = false;
  return device_status(c);
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
    for (int items : {256, 512, 1024})
      for (int slices : {1, 2, 4}) {
        rta_tuning tu{};
        tu.outputs_per_group = g;
        tu.tail_items = items;
        tu.bin_slices = slices;
        double us = 0;
        const int s2 = trial(schemes[best_s], tu, &us);
        if (s2 == RTA_E_DEVICE) return s2;
        if (s2 == RTA_OK && us < best_t) {
          best_t = us;
          bt = tu;
        }
      }
  }
  // stage 3: how the spectra are streamed, for that tiling
  for (int loads : {1, 2}) {
    rta_tuning tu = bt;
    tu.spectra_loads = loads;
    double us = 0;
    const int s2 = trial(schemes[best_s], tu, &us);
    if (s2 == RTA_E_DEVICE) return s2;
    if (s2 == RTA_OK && us < best_t) {
      best_t = us;
      bt = tu;
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

int rta_autotune_cached(const char* cache_path, double fs, int32_t block,
                        const rta_scheme* scheme, int32_t n_in, int32_t n_out,
                        const float* const* filters, const int64_t* lengths, int32_t spectra,
                        uint32_t flags, int32_t blocks, rta_tuning* best, double* best_us,
                        int32_t* from_cache) {
  if (cache_path == nullptr || best == nullptr || best_us == nullptr || blocks < 1) return RTA_E_ARG;
  std::vector<int> size, count;
  int st = validate(fs, block, scheme, n_in, n_out, filters, lengths, spectra, flags, size, count);
  if (st != RTA_OK) return st;
  const std::string key = tuning_key(fs, block, scheme, n_in, n_out, lengths, spectra, flags, blocks);
  rta_tuning t{};
  double us = 0;
  bool hit = cache_lookup(cache_path, key, &t, &us) && tuning_ok(&t);
  if (hit) {  // the cached scheme must still be a valid one for this shape
    std::vector<int> csize, ccount;
    const rta_scheme cs{t.n_tiers, t.size, t.count};
    hit = validate(fs, block, &cs, n_in, n_out, filters, lengths, spectra, flags, csize, ccount) == RTA_OK;
  }
  if (hit) {
    *best = t;
    *best_us = us;
    if (from_cache) *from_cache = 1;
    return RTA_OK;
  }
  st = rta_autotune(fs, block, scheme, n_in, n_out, filters, lengths, spectra, flags, blocks, &t, &us);
  if (st != RTA_OK) return st;
  *best = t;
  *best_us = us;
  if (from_cache) *from_cache = 0;
  return cache_append(cache_path, key, t, us);
}

int rta_serve_create(rta_ctx** out, double fs, int32_t block, const rta_scheme* scheme,
                     const rta_serve_config* cfg, int32_t spectra, uint32_t flags,
                     const rta_tuning* tuning) {
  if (out == nullptr) return RTA_E_ARG;
  *out = nullptr;
  if (cfg == nullptr || cfg->n_slots < 1 || cfg->n_out < 1 || cfg->max_taps < 1 ||
      cfg->max_taps > (int64_t(1) << 31) || cfg->arena_bytes < 0 || !(cfg->budget_bytes >= 0.0) ||
      !std::isfinite(cfg->budget_bytes))
    return RTA_E_ARG;
  if ((int64_t)cfg->n_slots * cfg->n_out > (1 << 20)) return RTA_E_ARG;
  if (!tuning_ok(tuning)) return RTA_E_ARG;
  if (flags & RTA_FLAG_NF3) return RTA_E_UNSUPPORTED;  // n_f = 2B only
  // the tiers are laid out for max_taps on every pair; no taps are read
  static const float dummy = 0.f;
  const int64_t np = (int64_t)cfg->n_slots * cfg->n_out;
  std::vector<const float*> f((size_t)np, &dummy);
  std::vector<int64_t> len((size_t)np, cfg->max_taps);
  std::vector<int> size, count;
  const int st = validate(fs, block, scheme, cfg->n_slots, cfg->n_out, f.data(), len.data(), spectra,
                          flags, size, count);
  if (st != RTA_OK) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || scratch_on(dev) == nullptr) {
    (void)hipGetLastError();
    return RTA_E_DEVICE;  // the scratch array of rta_serve_admit_noalloc
  }
  return create_ctx(out, fs, block, size, count, cfg->n_slots, cfg->n_out, f.data(), len.data(),
                    spectra, flags, tuning, cfg);
}

int rta_serve_admit(rta_ctx* c, const float* const* filters, const int64_t* lengths, int32_t* slot) {
  if (c == nullptr || filters == nullptr || lengths == nullptr || slot == nullptr) return RTA_E_ARG;
  if (c->serve == nullptr) return RTA_E_STATE;
  if (c->poisoned) return RTA_E_DEVICE;
  *slot = -1;
  for (int l = 0; l < c->L; ++l) {
    if (lengths[l] < 0 || lengths[l] > c->serve->cfg.max_taps) return RTA_E_ARG;
    if (lengths[l] > 0 && filters[l] == nullptr) return RTA_E_ARG;
  }
  return serve_admit(c, filters, lengths, slot, false);
}

int rta_serve_admit_noalloc(rta_ctx* c, const float* const* filters, const int64_t* lengths,
                            int32_t* slot) {
  if (c == nullptr || filters == nullptr || lengths == nullptr || slot == nullptr) return RTA_E_ARG;
  if (c->serve == nullptr) return RTA_E_STATE;
  if (c->poisoned) return RTA_E_DEVICE;
  *slot = -1;
  for (int l = 0; l < c->L; ++l) {
    if (lengths[l] < 0 || lengths[l] > c->serve->cfg.max_taps) return RTA_E_ARG;
    if (lengths[l] > kScratchTaps) return RTA_E_ARG;  // beyond the scratch array
    if (lengths[l] > 0 && filters[l] == nullptr) return RTA_E_ARG;
  }
  return serve_admit(c, filters, lengths, slot, true);
}

int rta_serve_release(rta_ctx* c, int32_t slot) {
  if (c == nullptr) return RTA_E_ARG;
  if (c->serve == nullptr) return RTA_E_STATE;
  if (slot < 0 || slot >= c->Q) return RTA_E_ARG;
  if (c->poisoned) return RTA_E_DEVICE;
  return serve_release(c, slot);
}

int rta_serve_query(rta_ctx* c, rta_serve_info* info, rta_slot_info* slots) {
  if (c == nullptr || info == nullptr) return RTA_E_ARG;
  if (c->serve == nullptr) return RTA_E_STATE;
  Serve* sv = c->serve;
  std::memset(info, 0, sizeof(*info));
  std::lock_guard<std::mutex> lk(sv->mu);
  info->n_slots = c->Q;
  for (size_t q = 0; q < sv->slots.size(); ++q) {
    const ServeSlot& sl = sv->slots[q];
    if (sl.state == RTA_SLOT_JOINING || sl.state == RTA_SLOT_LIVE) ++info->live;
    else if (sl.state == RTA_SLOT_FREE) ++info->free_slots;
    else ++info->draining;
    if (present(sl.state)) info->bytes_per_block += sl.hb + sl.xb;
    if (slots != nullptr) {
      rta_slot_info& o = slots[q];
      std::memset(&o, 0, sizeof(o));
      o.state = sl.state;
      const bool p = present(sl.state);
      o.start_block = p ? sl.start : -1;
      o.stop_block = p ? sl.stop : -1;
      o.free_block = p ? sl.free_at : -1;
      o.taps = p ? sl.taps : 0;
      o.bytes_per_block = p ? sl.hb + sl.xb : 0.0;
    }
  }
  const size_t eb = spectra_elem_bytes(c->dtype);
  for (int t = 0; t < c->n_tiers; ++t) {
    info->arena_bytes += sv->arena[t].capacity() * c->tier[t].P * (int64_t)eb;
    info->arena_used_bytes += sv->arena[t].used() * c->tier[t].P * (int64_t)eb;
  }
  info->budget_bytes = sv->cfg.budget_bytes;
  info->admitted = sv->admitted;
  info->rejected_slots = sv->rej_slots;
  info->rejected_memory = sv->rej_mem;
  info->rejected_budget = sv->rej_budget;
  info->plan_swaps = sv->swaps;
  return c->poisoned ? RTA_E_DEVICE : RTA_OK;
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
    case RTA_E_CAPACITY: return "no free slot or per-block bandwidth budget exceeded";
    default: return "unknown status";
  }
}

}  // extern "C"
