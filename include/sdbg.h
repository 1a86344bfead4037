/*
 * sdbg.h -- succinct de Bruijn graph (SdBG) construction on one MI355X GPU.
 *
 * Computes what Section 2 ("Methods") of Li et al., "MEGAHIT: an
 * ultra-fast single-node solution for large and complex metagenomics
 * assembly via succinct de Bruijn graph", defines:
 *
 *   sdbg_count_solid  every (k+1)-mer of the reads, on both strands, is
 *                     counted; those seen at least d times are solid; with
 *                     mercy enabled, the mercy-kmers are added (Section 2,
 *                     third paragraph).  Output: the edge set E sorted in
 *                     the SdBG edge order (colex order of the k-prefix, then
 *                     the last base; Section 2, second paragraph) with each
 *                     edge's count.
 *   sdbg_build        the SdBG arrays of an edge set: per-row label with a
 *                     minus flag (W), the last bit vector, F, the
 *                     edge-validity bit vector and the 2kt-bit vector of
 *                     zero-indegree vertex k-mers (Section 2, first
 *                     paragraph).
 *
 * All arithmetic is on integers; results are exact and do not depend on the
 * memory budget, the prefix length used for block-wise partitioning, or the
 * launch configuration.
 *
 * Encodings
 *   Bases A, C, G, T have codes 0, 1, 2, 3 (either case is accepted in
 *   reads).  Any other byte splits a read: no (k+1)-mer spans it.
 *   w = ceil(2(k+1)/64) 64-bit words per key.  The key of edge
 *   e = e[0..k] is the base-4 number with digits e[k-1], e[k-2], ..., e[0],
 *   e[k] (most significant first), stored right-aligned in w words, word 0
 *   most significant.  Ascending keys are the SdBG edge order.
 *   Rows of the graph: one per edge of E ("real"), one '$' row per vertex
 *   with no outgoing edge, and one dummy row per vertex v with no incoming
 *   edge (source '$' v[0..k-2], label v[k-1]).  Rows are ordered by source
 *   read from its last symbol to its first, then by label, with
 *   $ < A < C < G < T.
 *   W[i]   = label ($=0, A..T = 1..4) | 8 * minus[i]; minus[i] = 1 iff an
 *            earlier row has the same source[1..k-1] and the same non-$
 *            label.
 *   last   bit i = 1 iff row i is the last row of its source vertex.
 *   valid  bit i = 1 iff row i is a real edge.
 *   tip    bit i = 1 iff row i is a dummy row (t of them).
 *   mult[i] = count of a real row, 0 otherwise.
 *   F[c]   = number of rows whose source ends in a symbol < c, for
 *            c = $, A, C, G, T; F[5] = m.
 *   tip_seq: the t dummy rows' vertices v in row order, base j of the r-th
 *            at bits 2(k*r + j) (LSB first), ceil(2kt/64) words.
 *   Bit vectors are LSB-first 64-bit words: bit i of the vector is bit
 *   (i mod 64) of word i/64.
 *
 * Memory and ownership
 *   Inputs are borrowed for the duration of a call.  Output objects are
 *   allocated by the library, live in device memory (HBM) of the device
 *   current at the call, and are released with sdbg_free.  The *_to_host
 *   calls copy them into caller-provided host buffers.  Calls run on
 *   params->stream (a hipStream_t; NULL = the null stream) and return after
 *   the stream has completed the call's work.  Distinct calls may run
 *   concurrently from different host threads on different streams.
 *
 * Errors
 *   Every int-returning call returns SDBG_OK (0) or a negative code;
 *   sdbg_last_error() then returns a message for the calling thread.
 */
#ifndef SDBG_H
#define SDBG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDBG_OK 0
#define SDBG_E_INVAL (-1)        /* bad k, d, prefix_len or pointer */
#define SDBG_E_NOMEM (-2)        /* host allocation failed */
#define SDBG_E_NOMEM_DEVICE (-3) /* device memory or mem_budget cannot hold one block */
#define SDBG_E_HIP (-4)          /* HIP runtime error; message copied */
#define SDBG_E_BUSY (-5)         /* request queue full, or job already running */
#define SDBG_E_CANCELLED (-6)    /* job cancelled before it ran */

/* Reads: seq[offsets[i] .. offsets[i+1]) is read i; offsets[0] = 0 and the
 * offsets are non-decreasing.  on_device = 1: both pointers are device
 * pointers; 0: host pointers (copied to the device by the call). */
typedef struct sdbg_reads {
  const uint8_t *seq;
  const uint64_t *offsets;
  uint64_t n_reads;
  uint32_t on_device;
  uint32_t reserved;
} sdbg_reads;

/* k in [2, 127]; d >= 1 (solid threshold, 2 in the paper); mercy 0/1;
 * prefix_len l in [0, 8]: the key space is cut into 4^l blocks by the
 * length-l colex prefix of the k-mer and consecutive blocks that fit
 * mem_budget are processed together (Section 2, second paragraph; l = 0
 * disables the cut); mem_budget: bytes of device memory the key buffers of
 * one block group may use, 0 = 80% of free device memory. */
typedef struct sdbg_params {
  uint32_t k;
  uint32_t d;
  uint32_t mercy;
  uint32_t prefix_len;
  uint64_t mem_budget;
  void *stream;
} sdbg_params;

/* Edge set E: n keys (n*w words, ascending) and counts, in device memory.
 * n_mercy = edges added by the mercy rule (those with count < d);
 * n_occ = (k+1)-mer occurrences counted over both strands. */
typedef struct sdbg_edges {
  uint32_t k, w;
  uint64_t n, n_mercy, n_occ;
  uint64_t *keys;
  uint32_t *count;
} sdbg_edges;

/* SdBG arrays in device memory (F on the host). */
typedef struct sdbg_graph {
  uint32_t k, w;
  uint64_t m, t;
  uint8_t *W;        /* m bytes */
  uint64_t *last;    /* ceil(m/64) words */
  uint64_t *valid;   /* ceil(m/64) words */
  uint64_t *tip;     /* ceil(m/64) words */
  uint32_t *mult;    /* m */
  uint64_t F[6];
  uint64_t *tip_seq; /* tip_words words */
  uint64_t tip_words;
} sdbg_graph;

/* Count, filter and mercy (Section 2, third paragraph) -> *out. */
int sdbg_count_solid(const sdbg_reads *reads, const sdbg_params *params, sdbg_edges **out);

/* Allocation-free form of sdbg_count_solid, for callers that cannot
 * allocate device memory (code under stream capture, serving loops and
 * harnesses that forbid hipMalloc).  Computes exactly what
 * sdbg_count_solid computes, but every working buffer is carved out of one
 * fixed scratch array of SDBG_NOALLOC_SCRATCH_MB MiB per device, which the
 * device holds from the library's first use on it until the process ends,
 * and the edge set is written into the caller's buffers:
 *   keys_out   device, cap * w words (w = ceil(2(k+1)/64)), ascending keys;
 *   count_out  device, cap entries;
 *   *n_out     |E| (also when it exceeds cap: then SDBG_E_INVAL and the
 *              output buffers are left untouched, so the caller can retry
 *              with larger ones);
 *   *n_mercy_out, *n_occ_out, *scratch_peak_out (scratch bytes in use at
 *              the call's peak): as in sdbg_edges; each may be NULL.
 * reads, params: as for sdbg_count_solid; params->mem_budget is capped at
 * the scratch size.  An input whose bound on scratch use (from its read
 * lengths) exceeds the scratch, or that runs out of it, returns
 * SDBG_E_NOMEM_DEVICE before any kernel touches memory beyond the scratch.
 * Calls on one device share its scratch, which keeps the last call's
 * contents; they take turns (a per-device lock held until the call's
 * stream has completed), so concurrent calls in one process do not race.
 * Returns after params->stream has completed the call's work. */
#define SDBG_NOALLOC_SCRATCH_MB 256
int sdbg_count_solid_noalloc(const sdbg_reads *reads, const sdbg_params *params, uint64_t *keys_out,
                             uint32_t *count_out, uint64_t cap, uint64_t *n_out, uint64_t *n_mercy_out,
                             uint64_t *n_occ_out, uint64_t *scratch_peak_out);

/* SdBG arrays of an edge set (Section 2, first and second paragraphs).
 * Uses params->stream only (params may be NULL: null stream); the other
 * fields are ignored.  An edge set made by sdbg_edges_from_host is checked
 * first: SDBG_E_INVAL if its keys are not strictly ascending or have bits
 * above 2(k+1); edge sets the library computed are sorted by construction
 * and not checked again.  SDBG_E_INVAL also for an object this library did
 * not return. */
int sdbg_build(const sdbg_edges *edges, const sdbg_params *params, sdbg_graph **out);

/* Batched form: count (and, if graphs_out is not NULL, build) n_sets
 * independent read sets.  Results are identical to sdbg_count_solid and
 * sdbg_build on each set alone: edges_out[s] (and graphs_out[s]) receive
 * set s's objects, owned by the caller.  Consecutive sets whose keys fit
 * params->mem_budget (0 = 80% of free device memory) share every launch of
 * the partition, sort and count -- the paper sorts consecutive partitions
 * together in the same way (Section 2, second paragraph) -- so the number of
 * launches does not grow with the number of sets; a set larger than one
 * pass, and every set when mercy is on with d >= 2, runs on the single-set
 * path.  Sets may mix host and device reads.  On error no output is left
 * allocated and all entries are NULL. */
int sdbg_batch_run(const sdbg_reads *sets, uint64_t n_sets, const sdbg_params *params, sdbg_edges **edges_out,
                   sdbg_graph **graphs_out);

/* Launch parameters of the partition and sort, process-wide.  Results do
 * not depend on them.
 *   digit_bits      most key bits one refinement pass cuts, 4..8 (7)
 *   tile_shift      refinement pass tile = the key width's default tile
 *                   (3584, 2048, 1024, 1024 keys for w = 1..4) >> tile_shift,
 *                   0 or 1 (0)
 *   leaf_wg_per_cu  persistent workgroups per compute unit of the in-LDS
 *                   sort and count, 1..32 (16; fewer if fewer fit)
 *   leaf_cap_shift  largest segment sorted in LDS = the key width's default
 *                   (2048, 1024, 1024, 1024 keys for w = 1..4) >> leaf_cap_shift,
 *                   0 or 1 (0)
 *   first_bits      key bits of the first cut, which is taken straight from
 *                   the packed reads, 4..8 (6)
 *   mercy_shift     the mercy-kmer lookup table gets 2^mercy_shift times
 *                   fewer buckets than it is sized for, 0..8 (0); above 0
 *                   more lookups take the slower overfull-bucket path, which
 *                   is what this setting is for (testing that path)
 * (The autotuner varies the first four.) */
typedef struct sdbg_tune {
  uint32_t digit_bits;
  uint32_t tile_shift;
  uint32_t leaf_wg_per_cu;
  uint32_t leaf_cap_shift;
  uint32_t first_bits;
  uint32_t mercy_shift;
  uint32_t reserved[2];
} sdbg_tune;

int sdbg_tune_get(sdbg_tune *t);
/* NULL restores the defaults; SDBG_E_INVAL for a value out of range. */
int sdbg_tune_set(const sdbg_tune *t);

/* Autotuner: times reps (0 = 3) batched counts (sdbg_batch_run without
 * graphs) of the sample sets for each candidate value of one parameter at
 * a time (digit_bits 6..8, tile_shift 0..1, leaf_wg_per_cu 4..32,
 * leaf_cap_shift 0..1), keeps
 * the fastest, and leaves the best setting in effect (also copied to *best
 * if not NULL).  On error the previous setting is restored. */
int sdbg_autotune(const sdbg_reads *sets, uint64_t n_sets, const sdbg_params *params, uint32_t reps, sdbg_tune *best);

/* Served form: a request loop on the current device.  Jobs (a read set and
 * its parameters) are copied into pinned host memory at submit and queue in
 * FIFO order; max_jobs workers, each with its own stream, start the head of
 * the queue as soon as its device-memory footprint fits mem_budget next to
 * the running jobs, so jobs that arrive while others run join them on the
 * device (a job larger than the whole budget, or with a footprint above
 * 8 GiB, runs alone).  Each job runs
 * the single-call path (sdbg_count_solid, then sdbg_build if cfg->build),
 * so its results are identical to running it alone.  The device buffers of
 * finished jobs stay cached for the next ones (the memory-adaptive
 * construction reported in Section 3, under a shared budget). */
typedef struct sdbg_server_cfg {
  uint32_t max_jobs;   /* jobs running at once, at most 64; 0 = 4 */
  uint32_t queue_cap;  /* waiting jobs before submit returns SDBG_E_BUSY; 0 = 4096 */
  uint64_t mem_budget; /* device bytes shared by running jobs; 0 = 80% of free */
  uint32_t build;      /* 1: each job also builds the SdBG arrays */
  uint32_t reserved;
} sdbg_server_cfg;

/* Per-job record.  status: 1 waiting, 2 running, then SDBG_OK or the job's
 * error code; times in seconds since the server started; footprint = device
 * bytes reserved for the job at admission. */
typedef struct sdbg_job_stats {
  int32_t status;
  uint32_t reserved;
  double submit_s, start_s, end_s;
  uint64_t n_occ;
  uint64_t footprint;
} sdbg_job_stats;

typedef struct sdbg_server sdbg_server;

/* Device bytes the request loop reserves for a job of these reads and
 * parameters (host reads only): a bound on the job's peak use of the
 * library's device memory, used for admission. */
int sdbg_job_footprint(const sdbg_reads *reads, const sdbg_params *params, uint64_t *bytes);

/* Snapshot of the request loop: admission budget and the footprint bytes
 * of running jobs, waiting and running job counts, jobs not yet collected
 * by sdbg_server_poll, seconds since start. */
typedef struct sdbg_server_info {
  uint64_t budget, mem_in_use;
  uint32_t queued, running;
  uint64_t jobs;
  double uptime_s;
} sdbg_server_info;
int sdbg_server_state(sdbg_server *srv, sdbg_server_info *info);

/* Where a running job is, for diagnosis: the last kernel stage it entered,
 * what its worker waits on ("" if nothing: stream synchronisation, device
 * allocation, releasing cached device memory), and seconds since either
 * changed.  Empty strings for a job that is not running.  The strings are
 * static. */
int sdbg_server_trace(sdbg_server *srv, uint64_t job_id, const char **stage, const char **activity,
                      double *seconds);

/* Starts the workers (cfg may be NULL for defaults). */
int sdbg_server_start(const sdbg_server_cfg *cfg, sdbg_server **out);

/* Queues a job; reads must be host memory and are copied before the call
 * returns; params->stream is ignored.  SDBG_E_BUSY if the queue is full. */
int sdbg_server_submit(sdbg_server *srv, const sdbg_reads *reads, const sdbg_params *params, uint64_t *job_id);

/* Result of a job.  wait = 1 blocks until it has finished.  Returns 1 or 2
 * (waiting or running; only when wait = 0), else the job's final code:
 * SDBG_OK hands its edges (and graph, if built) to the caller -- NULL
 * pointers decline them and they are freed -- and forgets the job; an error
 * code also forgets it.  stats (may be NULL) receives its record.
 * SDBG_E_INVAL for an unknown id. */
int sdbg_server_poll(sdbg_server *srv, uint64_t job_id, int wait, sdbg_edges **edges, sdbg_graph **graph,
                     sdbg_job_stats *stats);

/* Cancels a waiting job (it finishes with SDBG_E_CANCELLED); SDBG_E_BUSY
 * if it is already running or finished. */
int sdbg_server_cancel(sdbg_server *srv, uint64_t job_id);

/* Cancels waiting jobs, waits for running ones, frees results nobody
 * polled, and releases the server.  No other call on srv may be in
 * progress or follow. */
int sdbg_server_stop(sdbg_server *srv);

/* Navigation of a graph on the device (Section 2, first paragraph: the
 * succinct representation is traversed through rank and select over W,
 * last and F).  sdbg_index_build makes rank directories over the graph's
 * arrays (about 2 bits per row; the index borrows the graph, which must
 * outlive it; release with sdbg_free).  A node is identified by the index
 * of its last row.  sdbg_navigate answers n queries rows[i] (device array)
 * into out (device array; n words, or n * ceil(2k/64) words for
 * SDBG_NAV_LABEL), on `stream`, and returns when they are done:
 *   SDBG_NAV_NODE      row -> its node
 *   SDBG_NAV_FORWARD   row -> node its edge enters (none for a '$' row)
 *   SDBG_NAV_BACKWARD  node -> node whose edge enters it (for a vertex with
 *                      no incoming edge: the dummy node before it; none for
 *                      a dummy node)
 *   SDBG_NAV_OUTDEG    node -> outgoing edges (0 for a '$' node)
 *   SDBG_NAV_INDEG     node -> incoming edges, dummy rows not counted
 *   SDBG_NAV_LABEL     node -> its k-mer v, base j at bits 2j (LSB-first
 *                      words); the k-mer of a vertex with no incoming edge
 *                      comes from tip_seq; all ones for a dummy node
 * "none" and out-of-range queries give all ones (UINT64_MAX).  Nodes are
 * given by any of their rows. */
#define SDBG_NAV_NODE 1
#define SDBG_NAV_FORWARD 2
#define SDBG_NAV_BACKWARD 3
#define SDBG_NAV_OUTDEG 4
#define SDBG_NAV_INDEG 5
#define SDBG_NAV_LABEL 6
typedef struct sdbg_index sdbg_index;
int sdbg_index_build(const sdbg_graph *g, const sdbg_params *params, sdbg_index **out);
int sdbg_navigate(const sdbg_index *index, int op, const uint64_t *rows, uint64_t n, uint64_t *out, void *stream);

/* Tip removal (Section 2, fourth paragraph, lists it among the cleaning
 * steps applied to each graph, without a definition; this is the reading
 * implemented).  On the graph as built (validity is not read, so the
 * result does not depend on earlier removals), a tip is
 *   forward:  a path v0 -> ... -> vj of 1 <= j <= max_len edges from a node
 *             with no incoming edge, through nodes of in- and out-degree 1
 *             (v0: out-degree 1), to a node vj with in-degree >= 2 (it joins
 *             the graph) or out-degree 0 (an isolated path);
 *   backward: the mirror image, from a node with no outgoing edge back
 *             through nodes of in- and out-degree 1 to a node with
 *             out-degree >= 2 or in-degree 0.
 * Every edge of every tip is removed at once by clearing its bit in
 * g->valid (in place, on `stream`; the call returns when it is done).
 * index must have been built on g (SDBG_E_INVAL otherwise).  *n_removed
 * (may be NULL) = valid bits cleared by this call.  max_len = 0 removes
 * nothing. */
int sdbg_remove_tips(sdbg_graph *g, const sdbg_index *index, uint32_t max_len, uint64_t *n_removed, void *stream);

/* Unitigs of a graph's valid edges (Section 2, fourth paragraph, and its
 * Fig. 1: contigs of one k feed the graph of the next; the paper gives no
 * construction, so this is the reading implemented).  Degrees count valid
 * edges only (g->valid after any cleaning).  A unitig is a maximal path
 * whose inner nodes have in-degree 1 and out-degree 1; every valid edge lies
 * on exactly one.  A unitig starts at an edge whose source node is not
 * (in 1, out 1); a cycle of such nodes starts at its smallest row.  Unitig
 * u, of len[u] edges, spells the k-mer of its first edge's source node and
 * then each edge's label (k + len[u] bases; for a cycle the last k repeat
 * the first k); mult[u] is the sum of its edges' mult.  Unitigs are listed
 * by the row of their first edge, ascending.  seq and offsets form a read
 * set on the device (sdbg_reads with on_device = 1), so the unitigs of one k
 * can be counted with the reads at the next.  index must have been built
 * on g (SDBG_E_INVAL otherwise).  The result lives in device memory;
 * release it with sdbg_free.  Working memory: about 40 bytes per row, 32
 * more if the valid edges hold cycles. */
typedef struct sdbg_unitigs {
  uint32_t k, reserved;
  uint64_t n;          /* unitigs */
  uint64_t n_cycles;   /* of which are cycles */
  uint64_t n_bases;    /* offsets[n] */
  uint64_t *first_row; /* n: row of the first edge */
  uint64_t *len;       /* n: edges */
  uint64_t *mult;      /* n: sum of mult over its edges */
  uint64_t *offsets;   /* n + 1: unitig u is seq[offsets[u] .. offsets[u+1]) */
  uint8_t *seq;        /* n_bases: 'A', 'C', 'G', 'T' */
} sdbg_unitigs;
int sdbg_unitigs_build(const sdbg_graph *g, const sdbg_index *index, sdbg_unitigs **out, void *stream);

/* Copies a unitig set to caller buffers of n, n, n, n + 1 words and n_bases
 * bytes; any pointer may be NULL to skip that array. */
int sdbg_unitigs_to_host(const sdbg_unitigs *u, uint64_t *first_row, uint64_t *len, uint64_t *mult,
                         uint64_t *offsets, uint8_t *seq);

/* Bubble merging and low-local-coverage removal (Section 2, fourth
 * paragraph, lists them with tip removal as the cleaning of each graph and
 * notes that the second suits the uneven depth of metagenomes; it defines
 * neither, so these are the readings implemented).  u must be the unitigs
 * of g's current valid edges (sdbg_unitigs_build after the last change to
 * g->valid; a unitig whose path no longer matches is skipped); index must
 * have been built on g.  Unitig u runs from s(u), the source node of its
 * first edge, to t(u), the node its last edge enters; cycles and unitigs of
 * more than max_len edges take part in neither call.
 *   sdbg_merge_bubbles: unitigs sharing s and t form a group; in a group of
 *     two or more, all but the one of highest mean multiplicity (mult / len,
 *     compared exactly as mult(a) * len(b) against mult(b) * len(a); ties
 *     to the smaller first row) are removed.
 *   sdbg_remove_low_coverage: the neighbouring edges of u are the valid
 *     edges other than its first and last that leave or enter s(u) or t(u);
 *     u is removed if it has one and its mean multiplicity is below
 *     ratio_permille / 1000 of theirs (exactly: mult(u) * count * 1000 <
 *     ratio_permille * len(u) * sum of their mult).
 * Every removal of a call is decided on g as given, then the valid bits of
 * the removed unitigs' edges are cleared (in place, on `stream`; the call
 * returns when it is done).  *n_removed (may be NULL) = valid bits cleared.
 * Take the unitigs again before the next call. */
int sdbg_merge_bubbles(sdbg_graph *g, const sdbg_index *index, const sdbg_unitigs *u, uint32_t max_len,
                       uint64_t *n_removed, void *stream);
int sdbg_remove_low_coverage(sdbg_graph *g, const sdbg_index *index, const sdbg_unitigs *u, uint32_t max_len,
                             uint32_t ratio_permille, uint64_t *n_removed, void *stream);

/* Union of two edge sets of the same k (e.g. the solid edges of the reads
 * and the edges of contigs): every key of either, ascending, with the two
 * counts summed where a key is in both (SDBG_E_INVAL if a sum does not fit
 * 32 bits).  n_mercy of the result is 0 and n_occ the sum of the two.
 * Runs on params->stream (params may be NULL). */
int sdbg_edges_union(const sdbg_edges *a, const sdbg_edges *b, const sdbg_params *params, sdbg_edges **out);

/* Cleaning of each graph of sdbg_multi_k: maximal lengths in edges as
 * multiples of k (0 skips the step) and the low-coverage ratio. */
typedef struct sdbg_clean_params {
  uint32_t tip_factor;       /* tips of at most tip_factor * k edges */
  uint32_t bubble_factor;    /* bubbles of unitigs of at most bubble_factor * k edges */
  uint32_t low_cov_factor;   /* unitigs of at most low_cov_factor * k edges ... */
  uint32_t low_cov_permille; /* ... below low_cov_permille / 1000 of their neighbours' mean */
} sdbg_clean_params;

/* Multiple k with contig feedback (Section 2, fourth paragraph, and Fig. 1:
 * graphs are built from a small k to a large one, each is cleaned of tips,
 * bubbles and low local coverage, and the contigs of one k go into the graph
 * of the next; the reading implemented): for each k of ks (n_k values,
 * ascending, each in [2, 127]):
 *   1. E = solid edges of the reads (sdbg_count_solid with params' d, mercy,
 *      prefix_len and mem_budget);
 *   2. from the second k on, E = E united with every (k+1)-mer of the
 *      previous k's unitigs, on both strands, with its count of occurrences
 *      in them (sdbg_count_solid of the unitigs with d = 1, no mercy, then
 *      sdbg_edges_union);
 *   3. the graph of E is built and cleaned: tips (sdbg_remove_tips), then
 *      bubbles (sdbg_merge_bubbles) and then low local coverage
 *      (sdbg_remove_low_coverage), each on the unitigs of the edges left,
 *      with the limits of *clean;
 *   4. the unitigs of the remaining valid edges are taken.
 * *out = the unitigs of the last k (release with sdbg_free).  stats (may be
 * NULL; 6 * n_k words): per k, the edges of E, the edges the unitigs added,
 * and the edges removed as tips, in bubbles and for low coverage, then the
 * unitigs.  Every intermediate object is released before the call
 * returns. */
int sdbg_multi_k(const sdbg_reads *reads, const uint32_t *ks, uint32_t n_k, const sdbg_params *params,
                 const sdbg_clean_params *clean, uint64_t *stats, sdbg_unitigs **out);

/* Burrows-Wheeler transform of a read set (Section 2, second paragraph:
 * the construction adapts CX1, whose core is sorting every suffix of every
 * read; the paper gives no details, so this is the multi-string BWT).  Read
 * r is followed by its own end marker $_r, smaller than every base, with
 * $_r < $_s for r < s.  Each read of length L has L + 1 suffixes (the last
 * is $_r alone); n = total bases + n_reads.  Sorted in that order, sa[i] is
 * the text position of the i-th suffix, where read r's suffix at offset j
 * (0 <= j <= L) is position offsets[r] + r + j, and bwt[i] is the character
 * before it in its read ('A', 'C', 'G', 'T', upper case), or '$' for a
 * suffix that starts its read.  Reads must hold only bases (either case;
 * SDBG_E_INVAL otherwise) and n + n_reads must stay below 2^32.  Runs on
 * params->stream (params may be NULL); the result lives in device memory
 * (release with sdbg_free). */
typedef struct sdbg_bwt {
  uint64_t n, n_reads;
  uint8_t *bwt; /* n characters */
  uint64_t *sa; /* n text positions */
} sdbg_bwt;
int sdbg_read_bwt(const sdbg_reads *reads, const sdbg_params *params, sdbg_bwt **out);

/* Copies a BWT to caller buffers of n bytes and n words (either may be NULL). */
int sdbg_bwt_to_host(const sdbg_bwt *b, uint8_t *bwt, uint64_t *sa);

/* Wraps host arrays (n*w key words ascending and unique, n counts) into a
 * library-owned device edge set, e.g. to build a graph from edges computed
 * elsewhere. */
int sdbg_edges_from_host(const uint64_t *keys, const uint32_t *count, uint64_t n, uint32_t k, sdbg_edges **out);

/* Copies an edge set to caller buffers of n*w words and n counts. */
int sdbg_edges_to_host(const sdbg_edges *edges, uint64_t *keys, uint32_t *count);

/* Copies graph arrays to caller buffers sized as in sdbg_graph; any pointer
 * may be NULL to skip that array. */
int sdbg_graph_to_host(const sdbg_graph *g, uint8_t *W, uint64_t *last, uint64_t *valid, uint64_t *tip, uint32_t *mult,
                       uint64_t *tip_seq);

/* Releases any object returned by the library; NULL is a no-op. */
void sdbg_free(void *obj);

/* Message of the calling thread's last failing call ("" if none). */
const char *sdbg_last_error(void);

/* Profiling.  While enabled (per host thread), each kernel a call launches
 * is bracketed by HIP events on the call's stream -- no synchronisation is
 * added -- and its elapsed time is read when the call completes.
 * sdbg_profile_get returns record i: the kernel's name (static string), its
 * duration in ms and the algorithmic bytes it reads and writes (the bytes
 * its inputs and outputs occupy, each counted once).  Returns SDBG_E_INVAL
 * if i is out of range. */
void sdbg_profile_enable(int on);
void sdbg_profile_reset(void);
uint32_t sdbg_profile_count(void);
int sdbg_profile_get(uint32_t i, const char **name, double *ms, uint64_t *bytes);

/* Releases the library's cached device memory (kept between calls to avoid
 * repeated allocation).  Objects not yet freed stay valid. */
void sdbg_trim(void);

/* Device memory of the library's caching pool on the current device:
 * bytes held by live buffers and outputs, the most held at any time since
 * the last call with reset_peak = 1 (which sets it to the current use), and
 * bytes cached for reuse.  Any pointer may be NULL. */
int sdbg_pool_stats(uint64_t *in_use, uint64_t *peak, uint64_t *cached, int reset_peak);

/* Failure injection for tests of the error paths: after `after` more pool
 * allocations on the current device succeed, the next one fails with
 * SDBG_E_NOMEM_DEVICE (once); a negative value disables it. */
int sdbg_fail_alloc_after(int64_t after);

#ifdef __cplusplus
}
#endif

#endif /* SDBG_H */
