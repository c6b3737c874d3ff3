/*
 * rta.h -- C ABI of librta: real-time multichannel partitioned convolution
 * (uniform and non-uniform partitioned overlap-save with a frequency-domain
 * delay line) on one AMD Instinct MI355X (gfx950).
 *
 * Operation (paper Sec. III-A Eq. 1-2): for Q input channels x_q and L output
 * channels,
 *
 *     y_l[n] = sum_{q<Q} sum_{j<n_h(q,l)} h_ql[j] * x_q[n-j]      (causal,
 *                                                     zero history before n=0)
 *
 * computed block by block: call k of rta_process() consumes input samples
 * [kB, (k+1)B) of every input and returns output samples [kB, (k+1)B) of
 * every output, with no added latency.  The filter matrix is split into
 * partitions whose spectra are multiplied with a frequency-domain delay line
 * of input spectra (Sec. IV steps 1-3, after Wefers); non-uniform schemes
 * (Sec. III-B, last paragraphs) add longer partitions for later filter
 * segments, whose delays are realized in the time domain.
 *
 * Conventions for every entry point:
 *   - Return value: RTA_OK (0) or a negative rta_status.  No exception or
 *     signal crosses the ABI; rta_strerror() names the code.
 *   - A context is used by one host thread at a time (serving contexts also
 *     accept one control thread, see rta_serve_create).  Distinct contexts
 *     are independent and may be used from different threads.
 *   - After RTA_E_DEVICE the context is poisoned: every later call except
 *     rta_query/rta_destroy returns RTA_E_DEVICE.
 *   - Argument validation happens before any HIP call, so RTA_E_ARG never
 *     touches the GPU.
 */
#ifndef RTA_H
#define RTA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rta_ctx rta_ctx;

typedef enum rta_status {
    RTA_OK = 0,
    RTA_E_ARG = -1,         /* invalid argument (NULL, size, scheme, dtype) */
    RTA_E_NOMEM = -2,       /* device or pinned host allocation failed      */
    RTA_E_RANGE = -3,       /* a filter spectrum exceeds the FP16 range      */
    RTA_E_DEVICE = -4,      /* a HIP runtime call failed; context poisoned   */
    RTA_E_STATE = -5,       /* call not valid in the context's current state */
    RTA_E_UNSUPPORTED = -6, /* valid request this build does not implement   */
    RTA_E_CAPACITY = -7     /* serving: no free slot, or the per-block
                               bandwidth budget would be exceeded           */
} rta_status;

/* Storage type of the filter spectra.  Input spectra, the multiply-
 * accumulate and both FFTs always run in FP32; the conversion to FP16/BF16
 * rounds to nearest-even and keeps subnormals. */
typedef enum rta_dtype { RTA_FP32 = 0, RTA_FP16 = 1, RTA_BF16 = 2 } rta_dtype;

/* rta_create() flags. */
#define RTA_FLAG_SPIKE   0x1u  /* NUPC: accumulate each later-tier frame in
                                  the single block after its FFT instead of
                                  spreading it over the frame's slack.     */
/* The n_f = 3 n_x variant (Sec. V, last paragraph): B-tap partitions with
 * 3B-point transforms (3B/2 packed bins per spectrum row, 1.5x the bytes of
 * n_f = 2B), input window [x_{n-2}, x_{n-1}, x_n], output = the last B of
 * the 3B samples.  Its point is the feedback convolution: the accumulated
 * spectrum of output l in block n is the transform of a frame whose last 2B
 * samples are [y_l(n-1), y_l(n)], exactly what B-tap feedback partitions
 * need, so rta_set_feedback's convolution takes those spectra as they are
 * instead of transforming y again (n_out fewer transforms per block).
 * Uniform partitions only (RTA_E_ARG otherwise); not for serving contexts
 * (RTA_E_UNSUPPORTED); rta_set_feedback then needs the same spectrum type as
 * the context and runs fused (RTA_E_UNSUPPORTED otherwise). */
#define RTA_FLAG_NF3     0x2u

/* Partition scheme (Sec. III-B: uniform and non-uniform partitioning).
 *   size[t]  partition length of tier t in samples; size[0] must equal the
 *            block length, every size is a power of two and a multiple of
 *            the block, and sizes strictly increase.
 *   count[t] number of partitions of tier t; count[n_tiers-1] == 0 means
 *            "as many as the longest filter needs".
 * Tier t covers filter taps [o_t, o_t + count[t]*size[t]) with o_0 = 0 and
 * o_{t+1} = o_t + count[t]*size[t].  A frame of tier t >= 1 (its input
 * samples complete at the end of one block) has s = (o_t + block - size[t])
 * / block blocks before its first output sample is due; its forward FFT
 * takes two of them, its inverse FFT two more (each transform runs as two
 * passes in consecutive blocks), so the scheme must satisfy s >= 5, i.e.
 * o_t >= size[t] + 4*block.  The multiply-accumulate is spread over
 * min(s - 4, size[t]/block - 1) blocks (1 with RTA_FLAG_SPIKE); with
 * o_t = 2*size[t] - block (s = size[t]/block) tiers with size[t] >=
 * 8*block qualify.  Other schemes return RTA_E_ARG.
 * A NULL scheme means uniform partitioning with size[0] = block, i.e. the
 * paper's UPOLS with n_k = n_x and n_f = 2 n_x (Sec. IV). */
typedef struct rta_scheme {
    int32_t n_tiers;
    const int32_t* size;
    const int32_t* count;
} rta_scheme;

#define RTA_MAX_TIERS 8

typedef struct rta_info {
    double fs;                    /* sampling rate given at creation       */
    double deadline_us;           /* block / fs in microseconds (Sec. I)   */
    int32_t block, n_in, n_out, n_tiers, spectra_dtype, n_phases;
    int32_t tier_size[RTA_MAX_TIERS];
    int32_t tier_count[RTA_MAX_TIERS];
    int64_t tier_offset[RTA_MAX_TIERS];
    int64_t blocks_done;          /* blocks processed since create/reset   */
    int64_t spectra_bytes;        /* filter spectra resident in HBM        */
    int64_t device_bytes;         /* all device memory held by the context */
    double  h_bytes_per_block;    /* filter-spectrum bytes streamed per
                                     block, averaged over the tier phases  */
    double  x_bytes_per_block;    /* input-spectrum (FDL) bytes read per
                                     block, counted once per (q, slot)     */
    double  io_bytes_per_block;   /* input block + output block bytes      */
    double  cmacs_per_block;      /* complex multiply-accumulates / block  */
    double  tail_bytes_per_block; /* algorithmic bytes of the multiply-
                                     accumulate kernel (partitions >= 1):
                                     their spectrum rows once plus their
                                     delay-line slots once per input       */
    int32_t grid;                 /* workgroups per block launch           */
    int32_t outputs_per_group;    /* outputs sharing one input-spectrum
                                     load in the multiply-accumulate       */
    int32_t rows_per_item;        /* partitions per workgroup work item    */
    int32_t poisoned;             /* 1 after RTA_E_DEVICE                  */
    int32_t feedback_paths;       /* 1 while rta_set_feedback paths are set */
    int32_t feedback_fused;       /* 1 if they run inside the block launch  */
    int32_t spectra_nontemporal;  /* 1 if the spectra are streamed with
                                     non-temporal loads (rta_tuning)       */
    int32_t fft_size;             /* first tier's real transform length:
                                     2*block, or 3*block with RTA_FLAG_NF3 */
    /* Host-side stages of rta_process() since create or rta_reset: calls,
     * per stage (input copy into pinned memory, kernel launch, wait for
     * the completion flag, output copy) the longest and the summed time in
     * microseconds, the slowest call (index since reset, total time), and
     * the waits that ran long enough (2 ms) to ask the stream for errors. */
    int64_t host_calls;
    double  host_max_us[4];
    double  host_sum_us[4];
    int64_t host_slowest_call;
    double  host_slowest_us;
    int64_t host_late_waits;
    int32_t bin_slices;           /* first-tier items per partition row,
                                     each over 1/bin_slices of the bins:
                                     rta_tuning's, or chosen when a long
                                     filter feeds few outputs (the partial
                                     slots per output group are capped so
                                     that a head adds them up while it
                                     transforms its window)                */
    int32_t max_group_slots;      /* the most partial slots one output
                                     group's head adds up per block        */
} rta_info;

/* Create a context.
 *   out      receives the context (set to NULL on failure).
 *   fs       sampling rate in Hz (> 0); used for deadline_us only.
 *   block    B, samples per call; power of two in [16, 4096].
 *   scheme   partition scheme (see rta_scheme) or NULL for UPOLS.
 *   n_in     Q >= 1 input channels;  n_out  L >= 1 output channels.
 *   filters  n_in*n_out host pointers, row-major [in][out]: filters[q*n_out+l]
 *            points to lengths[q*n_out+l] FP32 taps of h_ql.  A NULL pointer
 *            or a zero length means "no path".  The taps are copied during
 *            the call; the caller may free them on return.
 *   lengths  n_in*n_out tap counts (>= 0).
 *   spectra  rta_dtype of the stored filter spectra.
 *   flags    RTA_FLAG_* bits.
 * Allocates all device memory (spectra, delay lines, rings) on the current
 * HIP device and builds the filter spectra there.  Returns RTA_E_RANGE if
 * FP16 storage is requested and a spectrum value exceeds 65504 in
 * magnitude. */
int rta_create(rta_ctx** out, double fs, int32_t block,
               const rta_scheme* scheme, int32_t n_in, int32_t n_out,
               const float* const* filters, const int64_t* lengths,
               int32_t spectra, uint32_t flags);

/* Tiling of the kernels (performance only: every tiling gives the same
 * output up to FP32 rounding order).  Zero in any field selects the default.
 *   outputs_per_group  G in {1, 2, 4}: outputs sharing one input-spectrum
 *                      load in the multiply-accumulate (default 4 with later
 *                      tiers and at least 64 outputs, and with uniform
 *                      partitions, 16-bit spectra over 128 MB and at least
 *                      32 outputs; else 2 with at least 16 outputs, else 1).
 *   tail_items         target number of first-tier multiply-accumulate work
 *                      items per block (default 512).  With tail_rows unset,
 *                      items get at least as many partitions as keep every
 *                      output group's partial slots within what its output
 *                      workgroup adds up from registers (16 per thread,
 *                      256 / (bins per row) threads per bin), where the
 *                      block size and inputs allow it.
 *   tail_rows          partitions per first-tier item; overrides tail_items.
 *   tier_rows          partitions per later-tier item (default 16).
 *   bin_slices         S in {1, 2, 4, 8}: first-tier items cover 1/S of a
 *                      partition row's bins over S times more rows, so each
 *                      output group owns S times fewer partial sums for the
 *                      output workgroups to reduce (default: 2 for 16-bit
 *                      spectra with uniform partitions and at least 32
 *                      outputs, outside serving and n_f = 3B; else 1, or,
 *                      when the slot limit above has lengthened the items,
 *                      a power of two that brings them back to about 32 KB
 *                      of rows each; rta_info reports the choice).
 *   spectra_loads      how the multiply-accumulate streams the spectra:
 *                      1 = non-temporal loads, 2 = ordinary loads, 0 =
 *                      default (ordinary for uniform partitions, which
 *                      re-read every row every block, up to 384 MB of
 *                      spectra; non-temporal beyond that, with later tiers
 *                      and for serving contexts).
 * rta_autotune() also fills the scheme it selected (n_tiers, size, count). */
typedef struct rta_tuning {
    int32_t outputs_per_group;
    int32_t tail_items;
    int32_t tail_rows;
    int32_t tier_rows;
    int32_t bin_slices;
    int32_t n_tiers;
    int32_t size[RTA_MAX_TIERS];
    int32_t count[RTA_MAX_TIERS];
    int32_t spectra_loads;
} rta_tuning;

/* rta_create() with an explicit tiling (NULL: defaults).  The scheme fields
 * of `tuning` are ignored here; pass the scheme as `scheme`. */
int rta_create_tuned(rta_ctx** out, double fs, int32_t block,
                     const rta_scheme* scheme, int32_t n_in, int32_t n_out,
                     const float* const* filters, const int64_t* lengths,
                     int32_t spectra, uint32_t flags, const rta_tuning* tuning);

/* Autotuner.  Same arguments as rta_create(), except that a NULL scheme
 * means "choose one": the candidates are uniform partitioning and the
 * non-uniform schemes with partition ratios 8 (B, 8B, 64B) and 4 (B, 4B,
 * 16B, 64B), partitions up to 8192 or up to 2048 samples, and a first
 * (block-sized) tier of its minimum length or twice it; each later tier
 * starts at max(2 P_t - B, P_t + 4B) taps rounded up to whole partitions of
 * the tier before, limited to tiers the longest filter reaches.  For
 * every candidate scheme and tiling (G in {1, 2, 4} x tail_items in {256,
 * 512, 1024} x bin_slices in {1, 2, 4}, then spectra_loads 1 and 2 for the
 * best of those) a context is created, `blocks` blocks of zero input are run
 * through rta_process_device() after 16 warm-up blocks, and the mean block
 * time is measured with HIP events.  The fastest is written to *best and its
 * mean block time in microseconds to *best_us.  Takes one to a few seconds
 * per candidate, mostly building spectra; allocates and frees device memory
 * on the current device. */
int rta_autotune(double fs, int32_t block, const rta_scheme* scheme,
                 int32_t n_in, int32_t n_out, const float* const* filters,
                 const int64_t* lengths, int32_t spectra, uint32_t flags,
                 int32_t blocks, rta_tuning* best, double* best_us);

/* rta_autotune() behind a tuning cache at `cache_path`, a text file of one
 * JSON object per line.  The key covers the device (architecture name and
 * compute-unit count), fs, block, n_in, n_out, a hash of the filter lengths
 * (not the taps), spectra, flags, blocks and the scheme (or "auto2", the
 * current set of candidate schemes, for NULL).  On a hit with a valid entry, *best / *best_us come from the file
 * (*from_cache = 1; no device work); otherwise rta_autotune() runs and one
 * line is appended (*from_cache = 0).  from_cache may be NULL.  RTA_E_ARG if
 * the file cannot be appended to (the tuning is still returned).  One
 * writer per file at a time. */
int rta_autotune_cached(const char* cache_path, double fs, int32_t block,
                        const rta_scheme* scheme, int32_t n_in, int32_t n_out,
                        const float* const* filters, const int64_t* lengths, int32_t spectra,
                        uint32_t flags, int32_t blocks, rta_tuning* best, double* best_us,
                        int32_t* from_cache);

/* Process one block, host memory in and out, synchronously.
 *   in   [n_in][block] FP32 host array (row-major), read during the call.
 *   out  [n_out][block] FP32 host array, valid on return.
 * The input is copied into the context's pinned, device-mapped buffer and
 * one kernel is launched on the context's own stream.  Its output
 * workgroups read that buffer and write the output block straight into a
 * second pinned buffer over PCIe (no DMA copies); the last of them raises a
 * flag in pinned memory, on which the call spins before copying the output
 * to `out`.  The multiply-accumulate of partitions >= 2 for the next block,
 * in the same launch, keeps running after the call returns; the next call is
 * stream-ordered after it.  When that multiply-accumulate streams 32 MB or
 * more per block, its workgroups start only once this block's output
 * workgroups are done (they would slow them down), which shortens this
 * call at no cost to correctness.  Must not be interleaved with rta_process_device()
 * calls still in flight on another stream. */
int rta_process(rta_ctx* ctx, const float* in, float* out);

/* Process one block, device memory in and out, stream-ordered.
 *   d_in    [n_in][block] FP32 device array; d_out [n_out][block] FP32.
 *   stream  hipStream_t to launch on; NULL is HIP's null (default) stream.
 * Enqueues the block's kernel and returns without waiting; d_out is valid
 * once the stream has passed it.  Successive calls must be ordered on one
 * stream: the block index is kept on the host and passed to each launch, so
 * a launch captured into a graph and replayed would repeat the same block
 * (rta_graph_create below captures launches that read a device counter
 * instead). */
int rta_process_device(rta_ctx* ctx, const float* d_in, float* d_out,
                       void* stream);

/* Graph replay of runs of blocks (Sec. IV's per-block steps, device memory,
 * stream-ordered): the per-block launches of n_blocks consecutive blocks
 * captured once into a hipGraph and replayed, for callers that process
 * blocks in batches (offline rendering, throughput runs) and want to pay
 * one graph launch instead of n_blocks kernel launches.
 *   rta_graph_create: captures launch j (0 <= j < n_blocks) to read
 *     d_in + j*n_in*block ([n_blocks][n_in][block] FP32, device) and write
 *     d_out + j*n_out*block ([n_blocks][n_out][block]); the buffers must
 *     outlive the graph.  The kernels take their block index from a device
 *     counter (plus j) that the graph's last node advances by n_blocks, so
 *     replays need no host arguments.  n_blocks must be a multiple of
 *     rta_info.n_phases (the work lists repeat with that period; 1 for
 *     uniform partitions).  Allocates the 8-byte counter on first use and
 *     captures on a private stream; nothing runs on the device.
 *   rta_graph_launch: processes the context's next n_blocks blocks from the
 *     current contents of d_in into d_out, stream-ordered on `stream`
 *     (NULL: the null stream), exactly as n_blocks rta_process_device()
 *     calls would (bit-identical output).  Mixing with rta_process[_device]
 *     is allowed as long as the context's block index is a multiple of
 *     n_phases away from where the graph was captured (RTA_E_STATE
 *     otherwise); if other launches moved the index since the last replay, a
 *     one-thread kernel first sets the counter.  Block-timing spans do not
 *     see replays.
 *   rta_graph_destroy: NULL-safe; destroy graphs before their context.
 * RTA_E_UNSUPPORTED for serving contexts and for a feedback convolution in a
 * separate launch; rta_set_feedback after capture makes rta_graph_launch
 * return RTA_E_STATE.  RTA_E_DEVICE if capture or instantiation fails (the
 * context stays usable). */
typedef struct rta_graph rta_graph;
int rta_graph_create(rta_ctx* ctx, const float* d_in, float* d_out, int32_t n_blocks,
                     rta_graph** graph);
int rta_graph_launch(rta_graph* graph, void* stream);
int rta_graph_destroy(rta_graph* graph);

/* Feedback cancellation (Sec. III-A Eq. 3, Sec. V).  fb[q*n_out + l] points
 * to lengths[q*n_out + l] FP32 taps of f_ql, the estimated acoustic path
 * from output (loudspeaker) l to input (microphone) q -- row-major
 * [in][out] like the synthesis filters; NULL or length 0 means no path.
 * From then on block n's input is m_n - c_{n-1}: the feedback estimate
 * c = F * y, computed from the context's own output y by a second,
 * uniformly partitioned convolution (partition = block) on the GPU, is
 * subtracted from the next block of microphone samples.
 *
 * Where it runs, and what it costs on the latency path:
 *   - Fused (rta_info.feedback_fused = 1): when `spectra` equals the
 *     context's spectra type and the combined launch fits in LDS, the
 *     feedback convolution runs inside each block's single launch.  Its
 *     output workgroups (one per microphone, dispatched first) compute
 *     c_{n-1}; the synthesis output workgroups of block n reduce their own
 *     partial sums meanwhile, then WAIT for c_{n-1} before packing their
 *     input, and after emitting y(n) they transform it into the feedback
 *     delay line.  That wait is on rta_process's latency path: it adds the
 *     feedback heads' reduction, their partitions 0 and 1 over every output
 *     and one inverse FFT (measured 14-24 us per block for 1 -> 32 outputs
 *     and 0.1-5 s paths).  The wait is bounded: if it gives up, the block
 *     fails with RTA_E_DEVICE (from rta_process, or from the next
 *     rta_process_device / rta_query / rta_reset call) and the context is
 *     poisoned.
 *   - Separate: with another spectra type, the feedback convolution is a
 *     second launch on the same stream after each block.  It is off the
 *     latency path of the block that launches it, but the next block's
 *     launch is stream-ordered after it.
 *
 * Serving contexts (rta_serve_create): input slot q is microphone q and
 * f_ql its path from loudspeaker l.  The paths belong to the slot, not to
 * the source admitted into it, and stay in place across admissions and
 * releases.  While a slot is live its input is m_q - c_q (previous block);
 * while it is not live its input reads as zero, whatever m_q and c_q are
 * (its estimate is still computed, and unused).
 *
 * fb == NULL removes the paths.  Resets the context (as rta_reset; a serving
 * context keeps its live sources and frees released ones).  Taps are copied
 * during the call. */
int rta_set_feedback(rta_ctx* ctx, const float* const* fb, const int64_t* lengths,
                     int32_t spectra);

/* Test aid for the failure path of the fused feedback wait (above): bound
 * the synthesis workgroups' wait to max_polls polls (>= 1; default 2^24),
 * and with never_ready = 1 make the awaited count unreachable, so that every
 * fused block gives up after max_polls polls, reports RTA_E_DEVICE and
 * poisons the context.  Every kernel still runs to completion.  No device
 * call; RTA_E_ARG for max_polls < 1 or never_ready not in {0, 1}. */
int rta_test_feedback_wait(rta_ctx* ctx, int32_t max_polls, int32_t never_ready);

/* Zero all delay lines, input history, output rings and the block index, as
 * if the context had just been created.  Synchronous. */
int rta_reset(rta_ctx* ctx);

/* Fill *info with the context's geometry and counters (no device call). */
int rta_query(rta_ctx* ctx, rta_info* info);

/* Block timing (profiling aid).  Each block is one kernel launch (the heads
 * of this block, the later tiers' transform passes and the
 * multiply-accumulate of partitions >= 2 for the next block; with an
 * unfused feedback convolution, a second launch).  After rta_timing_enable(ctx, every) with every >= 1, the
 * blocks launched by rta_process() or rta_process_device() are timed in spans
 * of `every` consecutive blocks, the first span starting at the first block
 * launched after the call: one HIP event on the launch stream before a span's
 * first launch and one after its last.  With every = 1 that brackets each
 * block's kernels; a longer span also counts the gaps between back-to-back
 * launches but keeps the event packets, which delay the stream, off most
 * blocks.  rta_timing_read() waits for the recorded events and returns the
 * number of blocks in complete spans (0 if no span has completed) and their
 * summed time in milliseconds, then forgets them; a span still open is
 * dropped.  At most 65536 spans are kept.  rta_timing_enable(ctx, 0) stops
 * recording (a span still open is dropped); rta_reset drops an open span and
 * restarts the span grid at block 0; every < 0 is RTA_E_ARG. */
int rta_timing_enable(rta_ctx* ctx, int32_t every);
int rta_timing_read(rta_ctx* ctx, int64_t* blocks, double* block_ms);

/* Measurement aid, independent of any context: launch a streaming-read
 * kernel over the first floor(bytes/16)*16 bytes of device memory d_buf
 * (16-byte aligned) with `grid` workgroups of 256 threads.  Workgroup w reads
 * one contiguous chunk with the same 16-byte non-temporal loads as the
 * multiply-accumulate kernel and writes one float to d_sink[w] (d_sink holds
 * `grid` floats).  Stream-ordered on `stream` (NULL: HIP's null stream);
 * time it with events to get the attainable read bandwidth of this access
 * pattern.  Returns RTA_E_DEVICE if the launch fails. */
int rta_probe_read(const void* d_buf, int64_t bytes, int32_t grid, float* d_sink,
                   void* stream);

/* ---------------------------------------------------------------------------
 * Serving with continuous batching.
 *
 * A serving context is a context with n_slots inputs whose filters are not
 * fixed at creation: sources (a talker's or instrument's signal with its own
 * filters to every output, i.e. one row h_q. of Eq. 1's filter matrix) are
 * admitted into free slots and released while blocks keep streaming, and
 * all live sources are convolved and mixed into the n_out outputs by the same
 * one-launch-per-block path as rta_create()'s contexts (Eq. 2 over the live
 * slots).  rta_process() and rta_process_device() take [n_slots][block]
 * input; the rows of slots that are not live are ignored (read as zero).
 *
 * Admission (rta_serve_admit) is refused when
 *   - no slot is free                         -> RTA_E_CAPACITY,
 *   - the spectra do not fit in the HBM arena -> RTA_E_NOMEM,
 *   - the filter-spectrum and delay-line bytes streamed per block by all
 *     present sources plus the new one would exceed budget_bytes
 *                                              -> RTA_E_CAPACITY.
 * The new source's spectra are built on a separate stream into arena rows no
 * block reads, then the source joins at the next block boundary: the next
 * block launched reads its slot's input row (rta_serve_query reports that
 * block as start_block).  Work lists are double-buffered: the next block
 * switches to the new list, blocks in flight keep the old one.
 *
 * Release (rta_serve_release) stops the slot's input at the next block
 * boundary (stop_block); the slot keeps streaming its filters until every
 * delay line, history sample and partial sum it owns has returned to zero
 * (free_block), then becomes free and its arena rows are reused.
 * Its output tail (the filter's reverberation) is thus played out in full.
 *
 * Threads: one thread may run rta_process / rta_process_device while one
 * other thread calls rta_serve_admit / rta_serve_release / rta_serve_query;
 * the block thread only takes a short lock at each block boundary.
 * rta_set_feedback attaches per-slot feedback paths (see above); rta_reset
 * zeroes all state, keeps live sources and frees released ones.
 * ------------------------------------------------------------------------ */
typedef struct rta_serve_config {
    int32_t n_slots;       /* source slots (inputs), >= 1                   */
    int32_t n_out;         /* outputs, >= 1                                 */
    int64_t max_taps;      /* longest filter a source may bring, >= 1       */
    int64_t arena_bytes;   /* HBM for filter spectra; 0 = room for every
                              slot at max_taps on every output              */
    double  budget_bytes;  /* admission limit on spectrum + delay-line bytes
                              streamed per block by all present sources
                              (e.g. deadline x attainable bandwidth x a
                              safety factor); 0 = no limit                  */
} rta_serve_config;

typedef enum rta_slot_state {
    RTA_SLOT_FREE = 0,
    RTA_SLOT_JOINING = 1,   /* admitted; live from the next block           */
    RTA_SLOT_LIVE = 2,
    RTA_SLOT_LEAVING = 3,   /* released; input stops at the next block      */
    RTA_SLOT_DRAINING = 4   /* input stopped; tail still streaming          */
} rta_slot_state;

typedef struct rta_slot_info {
    int32_t state;              /* rta_slot_state                           */
    int32_t pad;
    int64_t start_block;        /* first block that read its input, or -1   */
    int64_t stop_block;         /* first block that ignored it, or -1       */
    int64_t free_block;         /* block from which the slot is free, or -1 */
    int64_t taps;               /* longest of its filters                   */
    double  bytes_per_block;    /* spectrum + delay-line bytes it streams   */
} rta_slot_info;

typedef struct rta_serve_info {
    int32_t n_slots, live, draining, free_slots;
    int64_t arena_bytes, arena_used_bytes;
    double  budget_bytes, bytes_per_block;  /* present sources            */
    int64_t admitted, rejected_slots, rejected_memory, rejected_budget;
    int64_t plan_swaps;         /* work-list switches at block boundaries   */
} rta_serve_info;

/* Create a serving context with no source admitted.  fs, block, scheme,
 * spectra, flags and tuning as for rta_create_tuned() (tuning may be NULL);
 * the scheme's tiers and the tiling are laid out for n_slots sources of
 * max_taps taps, so admissions never re-tile.  Allocates the spectra arena,
 * delay lines, partial sums and both work-list buffers up front. */
int rta_serve_create(rta_ctx** out, double fs, int32_t block,
                     const rta_scheme* scheme, const rta_serve_config* cfg,
                     int32_t spectra, uint32_t flags, const rta_tuning* tuning);

/* Admit a source.  filters[l] points to lengths[l] FP32 taps of its filter
 * to output l (n_out entries; NULL or length 0 = no path; every length
 * <= max_taps).  On success *slot receives the slot index whose input row
 * carries the source from the next block on.  Taps are copied during the
 * call, which returns after the spectra are built (milliseconds) without
 * waiting for the block thread.  Errors: see above; RTA_E_RANGE as for
 * rta_create. */
int rta_serve_admit(rta_ctx* ctx, const float* const* filters,
                    const int64_t* lengths, int32_t* slot);

/* rta_serve_admit() for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid it): the
 * same admission, but its filter-spectra build is staged in a fixed device
 * array that the library holds for the life of the process on each device
 * (5.5 MiB: up to 2^20 staged taps and 2^16 spectrum rows per batch), so
 * the call allocates nothing -- no hipMalloc, hipFree or allocating library
 * routine; it still copies the taps to the device and waits for the build.
 * Arguments and errors as rta_serve_admit(), plus RTA_E_ARG for a filter
 * longer than 2^20 taps (the array's limit) and RTA_E_DEVICE if the array's
 * device address could not be found.  The array is shared by every call on
 * one device: overlapping calls in one process are serialized by a lock
 * (each call clears the array's flag before use); concurrent calls that
 * bypassed the lock would race on it.  The output of the admitted source is
 * bit-identical to rta_serve_admit()'s. */
int rta_serve_admit_noalloc(rta_ctx* ctx, const float* const* filters,
                            const int64_t* lengths, int32_t* slot);

/* Release the source in `slot` (JOINING or LIVE; else RTA_E_STATE). */
int rta_serve_release(rta_ctx* ctx, int32_t slot);

/* Counters of a serving context, and per-slot state when `slots` is not
 * NULL (n_slots entries).  No device call.  RTA_E_STATE for a context
 * made by rta_create(). */
int rta_serve_query(rta_ctx* ctx, rta_serve_info* info, rta_slot_info* slots);

/* Release the context and all its memory.  NULL is accepted (no-op). */
int rta_destroy(rta_ctx* ctx);

/* Static, NUL-terminated description of a status code. */
const char* rta_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* RTA_H */
