/*
 * ewahthr.h -- C ABI of the MI355X (gfx950) T-of-N threshold library.
 *
 * Operation (Section 2, Formulation, of Kaser & Lemire, "Compressed bitmap
 * indexes: beyond unions and intersections"): given N bitmaps over the same r
 * rows and a threshold T, the result has row i set iff at least T of the N
 * inputs have row i set.  T = 1 is the union, T = N the intersection.  The
 * library extends the paper's range 1 <= T <= N to all T: T = 0 gives all ones
 * over the r rows, T > N gives all zeros, N = 0 gives all ones for T = 0 and
 * all zeros otherwise; an input listed twice counts twice.
 *
 * Bitmap format: EWAH with 64-bit words (Section 3.1, Compressed Bitmaps).  Row
 * i is bit (i mod 64) of uncompressed word floor(i / 64), least-significant
 * bit first (Section 3.1, Uncompressed Bitmaps).  A stream is a sequence of
 * marker words, each followed by K dirty ("literal") words; a marker holds the
 * fill bit in bit 0, the number L of fill words in bits 1..32 and K in bits
 * 33..63 (the paper defers the exact layout to the EWAH format paper and notes
 * 32-bit run counters; this is the reading adopted).  Inputs may be any
 * well-formed stream (split runs, empty markers, fill-valued literal words);
 * they must cover exactly U = ceil(r / 64) words and must not end inside a
 * literal run.  Padding bits past row r - 1 are ignored.  Outputs are always
 * canonical: every word equal to 0 or ~0 is a fill; a marker starts at word 0
 * and at every fill word that follows a literal or a fill of the other value;
 * literals attach to the preceding marker; trailing zero fills are explicit.
 *
 * All entry points return an ewah_status; on failure ewah_last_error() gives
 * a message (thread-local).  No exception crosses the ABI.  Memory ownership
 * is stated per call.  The library keeps one device (ewah_init) and is not
 * thread-safe: calls must come from one host thread at a time.
 */
#ifndef EWAHTHR_H
#define EWAHTHR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EWAH_OK = 0,
    EWAH_EINVAL = -1,   /* bad argument: null pointer, mismatched n_bits, size limits */
    EWAH_EFORMAT = -2,  /* malformed EWAH stream */
    EWAH_ENOMEM = -3,   /* host or device allocation failed */
    EWAH_ENOSPC = -4,   /* output capacity below ewah_output_bound() */
    EWAH_EDEVICE = -5   /* HIP runtime error, wrong device, or a device-side error flag */
} ewah_status;

/* A borrowed EWAH stream: n_words 64-bit words describing n_bits rows. */
typedef struct {
    const uint64_t* words;
    uint64_t n_words;
    uint64_t n_bits;
} ewah_view;

/* Library-owned registered bitmap (device-resident words plus indexes). */
typedef struct ewah_bitmap ewah_bitmap;

/* Per-bitmap catalog, computed at registration. */
typedef struct {
    uint64_t n_bits;
    uint64_t n_words;          /* compressed words (EWAHSize / 8) */
    uint64_t n_markers;
    uint64_t n_literals;       /* dirty words */
    uint64_t one_fill_words;   /* uncompressed words covered by fills of ones */
    uint64_t popcount;         /* number of rows set (|B_i|) */
    uint64_t run_count;        /* RunCount: runs of 0s and 1s over the r rows (Section 3.1) */
    uint64_t index_bytes;      /* device bytes of the locator, skip index and presence records */
} ewah_stats;

/* Selects the HIP device (must be gfx950) and allocates library state.  Idempotent. */
ewah_status ewah_init(int device);

/* Message of the last failed call on this thread ("" if none). */
const char* ewah_last_error(void);

/*
 * Registration (data loading, not part of a query; the paper likewise assumes
 * the bitmaps are in memory before a query, Section 2).  Validates the stream,
 * copies it to device memory and builds its index: the per-tile locator (for
 * every tile of 512 uncompressed words, the marker whose run covers the tile's
 * first word, with that marker word), the skip index (for every 64 compressed
 * words, which of them are markers and the position of the first one) and the
 * presence records (per tile, which 16-row quarters and which 8-row groups of each
 * word hold a one and how many quarters hold one, and which groups of 4 words hold
 * a dirty word or lie in a one-fill).  v->words is a host pointer if on_device == 0,
 * else a device pointer; it is only read during the call.  The call is
 * synchronous.  Limits: n_bits < 2^37 (U < 2^31 words).  EFORMAT if the stream
 * is malformed.  *out is owned by the caller until ewah_release().
 */
ewah_status ewah_register(const ewah_view* v, int on_device, ewah_bitmap** out);

/* Same for count bitmaps at once (one device allocation; the indexes are built on
 * up to 16 host threads); out[i] for v[i].  On failure nothing is registered and
 * the error names the lowest failing index. */
ewah_status ewah_register_many(const ewah_view* v, uint32_t count, int on_device, ewah_bitmap** out);

/* Frees a registered bitmap.  No query using it may still be in flight. */
void ewah_release(ewah_bitmap* b);

ewah_status ewah_get_stats(const ewah_bitmap* b, ewah_stats* out);

/* Device address of the registered stream (for tests and tools; read-only). */
const uint64_t* ewah_device_words(const ewah_bitmap* b);

/*
 * Upper bound on the canonical output length in words for inputs of
 * sum_input_words words in total over n_bits rows: 0 if n_bits = 0, else
 * min(U + 1, sum_input_words + 1).  U + 1: one word per position plus the
 * head marker.  sum + 1: every output word at a position p > 0 is charged to a
 * distinct input word at p (an output dirty word needs an input dirty word
 * there, since positions where every input is a fill give a fill; an output
 * marker needs an input dirty word or an input marker whose run starts there),
 * and the words at position 0 to the first marker and dirty word of an input,
 * plus one word of slack.  Queries need 1 <= N, so the N = 0 result (all ones
 * or all zeros over the rows) never needs a bound.
 */
uint64_t ewah_output_bound(uint64_t n_bits, uint64_t sum_input_words);

/*
 * T-of-N threshold of in[0..n-1] (Section 2: row i of the result is set iff at
 * least T of the n inputs have row i set; registered inputs, equal n_bits,
 * 1 <= n <= 4095; n = 0 is EINVAL since the row count would be undefined).
 * Writes the canonical EWAH result to out_words_dev (device memory, caller
 * owned, out_cap words) and its length to *out_n_words_dev (device memory).
 * out_cap must be >= ewah_output_bound(n_bits, sum of input n_words), else
 * ENOSPC without any device work.  The work is enqueued on hip_stream (a
 * hipStream_t, NULL = default stream) and the call returns without waiting;
 * inputs must stay registered until it completes.  Concurrent calls on
 * different streams are allowed.  A query of more tiles than there are
 * resident workgroups runs as a batch of one on the persistent kernel (same
 * result, still asynchronous).
 */
ewah_status ewah_threshold(const ewah_bitmap* const* in, uint32_t n, uint32_t T, uint64_t* out_words_dev,
                           uint64_t out_cap, uint64_t* out_n_words_dev, void* hip_stream);

/*
 * General symmetric function of the N input bits of every row (Section 2: the
 * threshold functions are a subset of the symmetric Boolean functions, which
 * include at-most-T and count-in-[T1, T2]; Section 3.2: a symmetric function is
 * determined by the number of ones among its inputs, XOR being the example;
 * Section 5.1: a counter-based method takes any function from [0, N] to the
 * Booleans).  Output row i is f[c_i], where c_i is the number of inputs with
 * row i set and f[0..n] is a host table (f_len = n + 1 bytes, 0 or non-zero),
 * read during the call only.  Any table is accepted: tables whose counts giving
 * 1 form at most 8 runs (at least T, at most T, exactly T, ranges, their
 * complements...) compare the bit-sliced counts with the runs' ends, odd and even
 * parity read the lowest count plane, and any other table is looked up per row
 * (one bit per count, staged in LDS).  Inputs, output buffers, bound, errors and
 * asynchrony as for ewah_threshold.
 */
ewah_status ewah_symmetric(const ewah_bitmap* const* in, uint32_t n, const uint8_t* f, uint32_t f_len,
                           uint64_t* out_words_dev, uint64_t out_cap, uint64_t* out_n_words_dev, void* hip_stream);

/*
 * Opt-threshold query (Section 3.3): T is not given; the query takes the
 * largest T in [0, n] whose T-of-N result has at least K rows (K = 1: the
 * largest T with a non-empty result, which is the largest row count, as
 * ScanCount finds it from its counters, Section 5.1) and returns that result.
 * *T_out (host memory) receives T; output buffers, bound and errors as for
 * ewah_threshold.  1 <= K <= n_bits, else EINVAL.  K = 1: one pass over the
 * inputs finds the largest count (tiles that cannot exceed the largest count
 * seen so far are skipped); K > 1: one pass builds the count histogram
 * (ewah_count_histogram) and T is the largest count whose suffix sum reaches
 * K.  The call is synchronous: it returns once T is known and the result has
 * been enqueued on hip_stream.
 */
ewah_status ewah_opt_threshold(const ewah_bitmap* const* in, uint32_t n, uint64_t K, uint64_t* out_words_dev,
                               uint64_t out_cap, uint64_t* out_n_words_dev, uint32_t* T_out, void* hip_stream);

/*
 * Count histogram (the counters of ScanCount, Section 5.1, summarised):
 * hist[c] = number of rows set in exactly c of the n inputs, c = 0..n.  hist
 * is host memory of n + 1 entries, owned by the caller.  Every opt-threshold
 * (Section 3.3) follows from it: the T-of-N result has sum over c >= T of
 * hist[c] rows.  Inputs as for ewah_threshold (1 <= n <= 4095, one n_bits);
 * no output bitmap is written.  Synchronous on hip_stream.  EINVAL for a null
 * or empty input list or a null hist.
 */
ewah_status ewah_count_histogram(const ewah_bitmap* const* in, uint32_t n, uint64_t* hist, void* hip_stream);

/*
 * As ewah_threshold, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * call allocates nothing.  Its per-call device state (tile-order ticket, input
 * slots, one 96-byte tile state per tile) lives in a static device array of
 * about 400 KB that each GPU holds until the process ends; queries of more than
 * 4096 tiles (n_bits > 2^27) are EINVAL.  Every call on one GPU shares that
 * array: calls that overlap (on different streams) race, calls on one stream
 * are ordered.  The input slots go to the device by a pageable copy from a
 * static host buffer, staged before the call returns.  Always one workgroup per
 * tile chained by look-back (never the batch of one); the default variant as for
 * ewah_threshold.  Inputs, outputs, bound, errors as for ewah_threshold.
 */
ewah_status ewah_threshold_noalloc(const ewah_bitmap* const* in, uint32_t n, uint32_t T, uint64_t* out_words_dev,
                                   uint64_t out_cap, uint64_t* out_n_words_dev, void* hip_stream);

/* As ewah_threshold with an explicit kernel variant (ewah_variant_code); the result is identical.
 * variant = 0 takes the default: the unary counter at T <= 2, else ewah_default_variant(). */
ewah_status ewah_threshold_v(const ewah_bitmap* const* in, uint32_t n, uint32_t T, uint64_t* out_words_dev,
                             uint64_t out_cap, uint64_t* out_n_words_dev, uint32_t variant, void* hip_stream);

/*
 * Kernel variant code: dense = 1 sends inputs whose dirty run covers a whole
 * tile through the register carry-save-adder tree; walk / litwalk (0..255)
 * are the longest compressed segment / dirty block handled by a single lane
 * before it is split across a wavefront.
 */
uint32_t ewah_variant_code(int dense, uint32_t walk, uint32_t litwalk);
/*
 * As ewah_variant_code, plus the per-row counter.  looped = 0: bit-sliced binary
 * counter with ripple-carry adds (the accumulator of BSTM, Section 5.3.1; with
 * dense = 1, whole-tile dirty runs go through a carry-save-adder tree instead);
 * looped = 1: unary saturating counter, one level per count 1..T (the Looped
 * recurrence, Section 6.2), taken when T <= bit length of N, else the binary
 * counter runs; dense is then ignored.  The result never depends on the code.
 */
uint32_t ewah_variant_code_ex(int dense, uint32_t walk, uint32_t litwalk, int looped);
/*
 * As ewah_variant_code_ex, plus the gate of the per-group count bounds (RBMrg's
 * second case, Section 6.4, applied to groups of words inside a tile that its run
 * counts do not settle): gate 0 counts them when T exceeds 1.1 times the mean
 * bound (the default), 1 always, 2 never, 3 when T exceeds 1.5 times the mean
 * bound.  Bounds only drop words that cannot reach T: the result never depends on
 * the code.
 */
uint32_t ewah_variant_code_full(int dense, uint32_t walk, uint32_t litwalk, int looped, uint32_t gate);
uint32_t ewah_default_variant(void);

/* ------------------------------------------------------------ batched path */

/* One query of a batch: indices into the batch's pool. idx is host memory, read during planning. */
typedef struct {
    const uint32_t* idx;
    uint32_t n;
    uint32_t T;
    uint64_t* out_words_dev;     /* device, caller owned, >= ewah_output_bound() words */
    uint64_t out_cap;
    uint64_t* out_n_words_dev;   /* device, caller owned */
    uint32_t variant;            /* 0 = library default */
} ewah_query;

typedef struct {
    uint32_t grid;          /* persistent workgroups, 0 = all that can be resident at once */
    int use_graph;          /* 1 = capture the batch's launches (bump, bounds pre-pass, persistent
                               kernel, scan, placement) into a hipGraph */
} ewah_batch_config;

typedef struct ewah_batch ewah_batch;

/*
 * Batches of threshold queries over one pool of bitmaps, as in the workloads
 * of Section 7.3 (thousands of queries, each over N bitmaps of one dataset),
 * each query with the meaning of ewah_threshold (Section 2).
 * Plans a batch: uploads the query table (inputs as pool indices, thresholds,
 * output pointers, variants) and, with use_graph, captures the launch into a
 * HIP graph.  Device memory per (query, tile) item: a 64-byte tile state, a
 * staging area of 520 words and 72 bytes of bounds pre-pass results.  pool[] must
 * stay registered while the batch exists.  All pool bitmaps must have the same
 * n_bits > 0.  Synchronous.
 */
ewah_status ewah_batch_plan(const ewah_bitmap* const* pool, uint32_t pool_n, const ewah_query* q, uint32_t nq,
                            const ewah_batch_config* cfg, ewah_batch** out);

/* Runs every query of the batch in one persistent launch on hip_stream (asynchronous). */
ewah_status ewah_batch_run(ewah_batch* b, void* hip_stream);

/* Replaces the per-query variants (nq entries, 0 = default).  Synchronous. */
ewah_status ewah_batch_set_variants(ewah_batch* b, const uint32_t* variants);

/* Sets the persistent grid size (workgroups); rebuilds the graph.  Synchronous. */
ewah_status ewah_batch_set_grid(ewah_batch* b, uint32_t grid);

/* Sets how many 64-word windows a wavefront decodes per batch of loads in the
 * persistent kernel (4..7, default 6; a kernel is built for each), a knob of the
 * autotuner; results never depend on it.  Rebuilds the graph.  Synchronous. */
ewah_status ewah_batch_set_win_batch(ewah_batch* b, uint32_t win_batch);

/* Turns the bounds pre-pass of the batch on (on != 0) or off, a knob of the autotuner;
 * results never depend on it.  With it, one wavefront per (query, tile) item of the
 * queries of at most 256 inputs evaluates the tile's count bounds from the presence
 * records (RBMrg's pruning, Section 5.2) in a launch of its own before the persistent
 * launch, which then takes only the tiles those bounds leave; without it, the
 * persistent launch evaluates them per tile.  Default: on for batches of at least
 * 65,536 items (many items keep the pre-pass's wavefronts busy; a short batch waits
 * for its widest query's).  Rebuilds the graph.  Synchronous. */
ewah_status ewah_batch_set_prepass(ewah_batch* b, int on);

void ewah_batch_free(ewah_batch* b);

/*
 * Reads and clears the device-side error flags (synchronises the device):
 * bit 0 = a tile's look-back wait gave up, bit 1 = a look-back ran past tile 0.
 * Either means the outputs of that launch are invalid.
 */
ewah_status ewah_device_errors(uint32_t* flags);

/* ------------------------------------------------------ learned selection */

/*
 * Per-query features (16 floats, row-major [nq][16]) computed on the device
 * from the registration catalog of the query's inputs: log2 N, log2 T, T/N,
 * log2(N - T + 1), mean / max / min / standard deviation of log2 density,
 * log2 of total and largest RunCount, log2 of total and largest compressed
 * size, dirty-word fraction, log2 r, (sum of densities) / T, and a constant 1.
 * These are the statistics the paper's hybrid assumes a database keeps
 * (compressed sizes, cardinalities, Section 8.1).  idx / offs / T are host
 * arrays: query q has inputs pool[idx[offs[q] .. offs[q+1])] and threshold
 * T[q].  feat_dev is device memory.  Asynchronous on hip_stream.
 */
ewah_status ewah_query_features(const ewah_bitmap* const* pool, uint32_t pool_n, const uint32_t* idx,
                                const uint32_t* offs, const uint32_t* T, uint32_t nq, float* feat_dev,
                                void* hip_stream);

/* Features of the queries of a planned batch (same definition). */
ewah_status ewah_batch_features(ewah_batch* b, float* feat_dev, void* hip_stream);

/*
 * Picks, for every query of the batch, the variant with the smallest
 * predicted cost: pred_dev is device memory [nq][n_arms] (e.g. the MLP's
 * predicted log-times), arm_codes[n_arms] (host) the variant codes.  The
 * choice is written into the batch's device query records (no host round
 * trip); a following ewah_batch_run uses it.  Asynchronous on hip_stream.
 */
ewah_status ewah_batch_select(ewah_batch* b, const float* pred_dev, uint32_t n_arms, const uint32_t* arm_codes,
                              void* hip_stream);

/* Copies the variant codes currently stored in the batch's device query records to host (synchronous). */
ewah_status ewah_batch_get_variants(ewah_batch* b, uint32_t* variants_host);

/*
 * Cost of every query inside the batch, the labels of the learned selector
 * (trained on timings the method itself generates; the paper takes the minimum
 * of repeated runs as the true time, Section 7.5): runs the batch reps times
 * (eager launches, the batch's grid and variants) and writes, per query, the
 * minimum over the runs of the time the workgroups spent on its tiles, in
 * microseconds (device wall clock), into busy_us[nq] (host).  The bounds
 * pre-pass's wavefronts count at the share of a CU they hold relative to a
 * workgroup of the tile routine.  A persistent launch takes about the sum of
 * these times divided by its grid.  Synchronous.
 */
ewah_status ewah_batch_time_queries(ewah_batch* b, uint32_t reps, float* busy_us, void* hip_stream);

/* --------------------------------------------------------------- selector */

/*
 * The variant selector as a library object: a learned cost model (an FP32 MLP
 * predicting every variant's log-time from the 16 query features; machine-
 * learned algorithm selection is the paper's future work, Section 9) and the
 * paper-style rule set (per variant a running-time model of the forms of
 * Section 8.1 -- compressed size, size times ln N, N times tiles, T times size,
 * dirty words -- fitted by least squares; hybrid H takes the smallest estimate,
 * Section 8.2).  The variant with the smallest prediction is taken; selection
 * never changes a result.
 */
typedef struct ewah_selector ewah_selector;
enum { EWAH_SELECT_MLP = 0, EWAH_SELECT_RULES = 1 };

/* Training settings; zero fields take the defaults (80 epochs, batch 1024, lr 2e-3, seed 1). */
typedef struct {
    uint32_t epochs;
    uint32_t batch;
    float lr;
    uint64_t seed;
} ewah_train_config;

/*
 * Loads a model file (JSON object: "arm_codes" [K], "mu" [16], "sigma" [16],
 * "params_raw" [P], optionally "params_folded" [P] and "rules_coef" [5][K]; P =
 * ewah_mlp_num_params(K); other keys are ignored) and uploads the network.
 * EFORMAT if a key is missing or malformed.  *out is owned by the caller until
 * ewah_selector_free().  Host only: the device copy of the network is made by the
 * first prediction (ewah_init must have been called by then).
 */
ewah_status ewah_selector_load(const char* path, ewah_selector** out);
/* Writes the model in the format ewah_selector_load reads. */
ewah_status ewah_selector_save(const ewah_selector* s, const char* path);
void ewah_selector_free(ewah_selector* s);
uint32_t ewah_selector_num_arms(const ewah_selector* s);
/* Variant codes of the arms (K entries, host). */
ewah_status ewah_selector_arm_codes(const ewah_selector* s, uint32_t* codes);

/*
 * Trains a selector on n labelled queries: feat [n][16] (host; the features of
 * ewah_query_features), log2_time [n][n_arms] (host; log2 of each arm's measured
 * time in microseconds, e.g. from ewah_batch_time_queries), arm_codes [n_arms].
 * The features are standardised over the set (the constant feature stays 1);
 * the targets are each arm's log-time minus the query's mean over the arms.
 * The network is trained on the GPU by the library's forward, backward and
 * Adam kernels (mean squared error, mini-batches shuffled by a counter-based
 * SplitMix64 stream of cfg->seed); the standardisation is then folded into the
 * first layer.  The rule set is fitted on the same labels.  Synchronous; *out is
 * owned by the caller.  EINVAL for empty sets, more than 16 arms or non-finite labels.
 */
ewah_status ewah_selector_train(const float* feat, const float* log2_time, uint32_t n, uint32_t n_arms,
                                const uint32_t* arm_codes, const ewah_train_config* cfg, ewah_selector** out);
/* Training loss (mean squared error) of the last epoch's last mini-batch. */
float ewah_selector_train_loss(const ewah_selector* s);

/* pred_dev [n][K] = predicted cost of every arm for feat_dev [n][16] (device memory, asynchronous):
 * mode EWAH_SELECT_MLP (relative log2-time) or EWAH_SELECT_RULES (microseconds). */
ewah_status ewah_selector_predict(const ewah_selector* s, int mode, const float* feat_dev, uint32_t n, float* pred_dev,
                                  void* hip_stream);

/*
 * Features, prediction and per-query argmin for a planned batch, all on the device
 * (no host round trip): the chosen variant codes land in the batch's query records and
 * the next ewah_batch_run uses them.  The features of a batch do not change, so one
 * call per plan is enough.  Asynchronous on hip_stream.
 */
ewah_status ewah_batch_select_model(ewah_batch* b, const ewah_selector* s, int mode, void* hip_stream);

/*
 * FP32 multilayer perceptron 16 -> 64 -> 64 -> n_out (ReLU), the cost model
 * of the selector.  Parameters live in device memory; layout (floats):
 * W1[16][64], b1[64], W2[64][64], b2[64], W3[64][n_out], b3[n_out].
 * Initialisation: He-uniform from a counter-based SplitMix64 stream of seed.
 */
typedef struct ewah_mlp ewah_mlp;
ewah_status ewah_mlp_create(uint32_t n_out, uint64_t seed, ewah_mlp** out);
void ewah_mlp_free(ewah_mlp* m);
uint64_t ewah_mlp_num_params(uint32_t n_out);
ewah_status ewah_mlp_get_params(const ewah_mlp* m, float* host, uint64_t n);
ewah_status ewah_mlp_set_params(ewah_mlp* m, const float* host, uint64_t n);   /* also resets Adam state */
/* y_dev[batch][n_out] = network(x_dev[batch][16]) (device memory, asynchronous) */
ewah_status ewah_mlp_forward(ewah_mlp* m, const float* x_dev, uint32_t batch, float* y_dev, void* hip_stream);
/*
 * Gradient of the loss mean over (sample, output) of (y - t)^2 with respect
 * to every parameter, into grad_dev (device, num_params floats, overwritten),
 * loss into *loss_dev (device).  Asynchronous.
 */
ewah_status ewah_mlp_grad(ewah_mlp* m, const float* x_dev, const float* t_dev, uint32_t batch, float* grad_dev,
                          float* loss_dev, void* hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; loss before the step into *loss_dev. */
ewah_status ewah_mlp_train_step(ewah_mlp* m, const float* x_dev, const float* t_dev, uint32_t batch, float lr,
                                float* loss_dev, void* hip_stream);
const char* ewah_mlp_last_error(void);

/* Number of compute units of the device (0 before ewah_init). */
uint32_t ewah_num_cus(void);

#ifdef __cplusplus
}
#endif
#endif /* EWAHTHR_H */
