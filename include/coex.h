/*
 * coex.h — C ABI of libcoex, a chunked speculative finite-automaton scan of
 * DNA sequences on AMD Instinct MI355X (gfx950).
 *
 * The operations follow Memeti & Pllana, "Analyzing large-scale DNA Sequences
 * on Multi-core Architectures" (CSE 2015):
 *   - the problem (Section II): text T[1..n] over {A,C,G,T}, a pattern set;
 *     find every occurrence, overlapping ones included;
 *   - the automaton (Section II): (Q, Sigma, delta, q0, F) with a complete
 *     transition table, built by Aho-Corasick with the failure links folded
 *     into explicit transitions (Section III.B.1, Fig. 2), or from a regular
 *     expression (Table IV syntax);
 *   - the scan (Section III, Algorithm 1): the text is cut into chunks; every
 *     chunk is scanned speculatively from its possible starting states, the
 *     redundant runs stop at the converging point, and a join links each
 *     chunk's last state to the next chunk's first state; the counts are fixed
 *     up at the converging point.  Results equal one sequential scan from q0.
 *
 * Conventions shared by every call
 *   - Every call returns an int status: COEX_OK (0) or a negative COEX_E*
 *     code; coex_strerror() names it.  No exception crosses the ABI.  On an
 *     error, output buffers are left untouched unless stated otherwise.
 *   - Handles (coex_dfa*) are created by the coex_compile_* / from_table calls,
 *     are immutable afterwards, may be shared between threads, and are
 *     released by coex_dfa_free().  The library keeps a device copy of the
 *     tables per GPU, made on first use and freed with the handle.
 *   - Sequence and result pointers named *_dev are device pointers (HIP
 *     memory on the current device) owned by the caller; the library never
 *     frees them.  Other pointers are host pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     queued on it asynchronously unless the call says it synchronises.
 *     Calls on the same stream may reuse one library workspace; calls that
 *     run concurrently must use different streams.
 *   - Alphabet: A,C,G,T in either case.  In a sequence every other byte (N,
 *     IUPAC codes, newlines, ...) resets the automaton to q0, so no match ends
 *     on or spans such a byte.  Patterns must be non-empty over A,C,G,T.
 *   - Match end positions are 0-based indices of the last base of the match,
 *     reported in ascending order, ties by ascending pattern id.
 */
#ifndef COEX_H
#define COEX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define COEX_OK 0
#define COEX_EINVAL (-1)      /* bad argument (NULL where not allowed, bad sizes, misaligned pointer) */
#define COEX_EALPHABET (-2)   /* pattern character outside A,C,G,T, or an empty pattern */
#define COEX_ETOOBIG (-3)     /* the automaton has more states than the device tables can index (4096) */
#define COEX_ENOMEM (-4)      /* host or device allocation failed */
#define COEX_ECAPACITY (-5)   /* result buffer too small; the required size is reported */
#define COEX_EDEVICE (-6)     /* a HIP runtime call failed */
#define COEX_EUNSUPPORTED (-7)/* option combination not supported */
#define COEX_ESYNTAX (-8)     /* regular expression syntax error, or it matches the empty string */
#define COEX_EINTERNAL (-9)   /* a device-side consistency check failed */
#define COEX_ESCRATCH (-10)   /* coex_count_noalloc: the call needs more than its static scratch array */
#define COEX_ENOTRESIDENT (-11) /* coex_count_noalloc: the automaton's tables are not yet on this device */

/* ------------------------------------------------------- sequence formats */
#define COEX_ENC_BYTE 0  /* one ASCII byte per base */
#define COEX_ENC_2BIT 1  /* A=0 C=1 G=2 T=3, base i in bits 2*(i%4).. of byte i/4;
                            N mask: bit i%8 of byte i/8 set = base i is N (its code is ignored) */

typedef struct coex_dfa coex_dfa;

/* A sequence resident in device memory (the text T[1..n] of Section II).
   The sequence is the n_bases bases that follow the first `first_base` bases
   of the buffers; positions reported for it count from its own first base.
   COEX_ENC_BYTE: `bases` may have any address (a sequence that starts after a
   FASTA header line, say); the scans read from the 16-byte boundary at or
   below it.  COEX_ENC_2BIT: `bases` and `n_mask` must be 16-byte aligned;
   first_base selects the starting base (any value).  n_mask may be NULL for
   COEX_ENC_2BIT (no N) and is ignored for COEX_ENC_BYTE.  Batches
   (coex_batch_*) take 16-byte aligned buffers with first_base = 0. */
typedef struct {
  const void* bases;
  const uint8_t* n_mask;
  uint64_t n_bases;
  int32_t encoding;
  uint64_t first_base;
} coex_seq;

/* Scan options; 0 in any field lets the planner choose.
   chunk:    bases per chunk (any value >= 1; the planner uses multiples of 512)
   width:    lanes given to one chunk's speculative runs (1..64, power of two);
             a chunk with more possible starting states than `width` is run
             from all of them to its end instead
   lookback: k, the number of bases before a chunk used to narrow its possible
             starting states (1 = the paper's single last symbol; 1..8)
   step:     symbols per table lookup in the main loop (1, 2 or 3; 2 needs at
             most 1024 states, 3 at most 1023: five three-symbol lookups and
             one one-symbol lookup per 16 bases)
   flags:    COEX_FLAG_CHECK: synchronise the stream at the end of the call and
             return COEX_EINTERNAL if a device-side consistency check failed;
             COEX_FLAG_TIME: time the scan kernel (coex_profile)
   chains:   chunks one lane walks at once, their table lookups interleaved
             so that several dependent chains of reads are in flight (1 or 2;
             2 needs step 2 or 3) */
typedef struct {
  uint32_t chunk;
  uint32_t width;
  uint32_t lookback;
  uint32_t step;
  uint32_t flags;
  uint32_t chains;
} coex_opts;

#define COEX_FLAG_CHECK 1u
#define COEX_FLAG_TIME 2u  /* record HIP events around the scan kernel (see coex_profile) */
#define COEX_FLAG_GRAPH 4u /* batches: capture the launch sequence in a HIP graph at the first run
                              and replay it on later runs */

/* Facts about a compiled automaton. */
typedef struct {
  uint32_t n_states;    /* |Q| */
  uint32_t n_patterns;  /* number of pattern ids (counts arrays have this length) */
  uint32_t n_accepting; /* |F| */
  uint32_t q0;          /* start state */
  uint32_t sync_depth;  /* smallest d such that any two states reach the same state after any d
                           symbols; 0xFFFFFFFF if no such d exists */
  uint32_t max_out;     /* largest number of patterns ended by one state */
  uint32_t max_pss[9];  /* max_pss[k] = largest number of possible starting states after a
                           k-base lookback (k = 1..8); max_pss[0] = n_states */
} coex_dfa_info_t;

/* ------------------------------------------------------------ automata */

/* Aho-Corasick automaton of `n` patterns (Section II; failure links folded
   into a complete table, Section III.B.1).  Pattern id = index in `kmers`.
   Duplicates are allowed and each id counts every occurrence.  Patterns may
   have different lengths.  Errors: EINVAL (n == 0 or NULL), EALPHABET,
   ETOOBIG, ENOMEM. */
int coex_compile_kmers(const char* const* kmers, uint32_t n, coex_dfa** out);

/* Search automaton of one regular expression R (Table IV syntax): alternation
   '|', grouping '()', classes '[ACG]', '.', and the repeats '?', '*', '+',
   '{m}', '{m,}', '{m,n}'.  The automaton recognises Sigma* R and is minimised;
   it has one pattern (id 0), reported once per end position at which some
   match of R ends.  Errors: EINVAL, ESYNTAX (also for an R that matches the
   empty string), ETOOBIG, ENOMEM. */
int coex_compile_regex(const char* regex, coex_dfa** out);

/* An automaton given as a table (Section II quintuple): delta[s*4 + c] is the
   successor of state s on symbol c (A,C,G,T = 0..3); out_offsets[s] ..
   out_offsets[s+1] index into out_ids the pattern ids that end at state s
   (a state with an empty set is not final).  Host arrays, copied.  State
   numbering is kept in every output.  Errors: EINVAL (a successor or id out
   of range, offsets not non-decreasing, a repeated id within a state),
   ETOOBIG, ENOMEM. */
int coex_dfa_from_table(const uint32_t* delta, uint32_t n_states, uint32_t q0, const uint32_t* out_offsets,
                        const uint32_t* out_ids, uint32_t n_patterns, coex_dfa** out);

int coex_dfa_info(const coex_dfa* dfa, coex_dfa_info_t* info);

/* Copies the automaton out as plain host arrays: delta[n_states*4],
   out_offsets[n_states+1], out_ids[out_offsets[n_states]] (ascending within a
   state).  Any pointer may be NULL to skip that array. */
int coex_dfa_export(const coex_dfa* dfa, uint32_t* delta, uint32_t* out_offsets, uint32_t* out_ids);

void coex_dfa_free(coex_dfa* dfa);

/* ------------------------------------------------------------ scans */

/* Per-pattern match counts of `dfa` over `seq` (Section III, Algorithm 1:
   chunks, possible starting states, converging point, join, fix-up).
   counts_dev: uint64[n_patterns] device buffer, overwritten.
   Asynchronous on `stream`.  The kernels check their own consistency (every
   recount reaches the state the scan found, every true first state is a
   candidate); with COEX_FLAG_CHECK the call waits and returns EINTERNAL on a
   failure, without it the failure is kept for coex_errors_async.
   Errors: EINVAL, ENOMEM, EDEVICE. */
int coex_count(const coex_dfa* dfa, const coex_seq* seq, uint64_t* counts_dev, const coex_opts* opts,
               void* stream);

/* coex_count for callers that cannot allocate device memory: code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
   arguments, plan, kernels and results as coex_count, but the call makes no
   hipMalloc, hipFree or other allocating call: its scratch (per-chunk
   converging points, states and counts, the fix-up list and, for automata
   that can leave a chunk unconverged, the candidate maps) lives in one static
   device array of 64 MiB per GPU (its last 256 bytes keep the calls'
   consistency failures for coex_errors_async), held from library load to
   process exit.
   That covers every planner-chosen chunking of an automaton whose chunks
   always converge (about 36 bytes per chunk); a call whose plan needs more
   returns ESCRATCH before launching anything.  Device counters are cleared by
   a kernel at the start of every call, so no state carries over from the
   previous call, but every call on one GPU shares that GPU's array: calls
   that overlap on one GPU (other streams, other threads) race and must be
   serialised by the caller.  The automaton's tables must already be on the
   current device (any earlier coex_count, coex_find or coex_count_chunks on
   that device puts them there), else ENOTRESIDENT.  COEX_FLAG_TIME is not
   supported (EUNSUPPORTED); COEX_FLAG_CHECK synchronises as for coex_count.
   Errors: EINVAL, ENOTRESIDENT, ESCRATCH, EUNSUPPORTED, EDEVICE. */
int coex_count_noalloc(const coex_dfa* dfa, const coex_seq* seq, uint64_t* counts_dev, const coex_opts* opts,
                       void* stream);

/* End positions of every match ("count and extract", Section III.A):
   pos_dev int64[capacity] and pattern_dev uint32[capacity] (may be NULL)
   receive the matches in ascending end position, ties by pattern id.
   *n_found (host) receives the number of matches.  One pass over the
   sequence: the scan appends each match as it is found (end position and
   pattern id in one key, so at most 2^24 pattern ids and 2^40 bases; beyond
   that, or with opts->chains = 2, a second pass writes them in order);
   the stream is synchronised once to read the total, then the keys are
   sorted on the stream.  If the total exceeds `capacity`, *n_found holds the
   required size, ECAPACITY is returned and the contents of pos_dev and
   pattern_dev are unspecified. */
int coex_find(const coex_dfa* dfa, const coex_seq* seq, int64_t* pos_dev, uint32_t* pattern_dev,
              uint64_t capacity, uint64_t* n_found, const coex_opts* opts, void* stream);

/* Counts and end positions from one scan (both results of "count and
   extract", Section III.A): coex_find, then counts_dev uint64[n_patterns]
   (device, caller-owned) from the matches found, one small kernel that
   reads the pattern ids back (one-pattern automata: the number of matches).
   The counts equal coex_count's.  pattern_dev is required when the
   automaton has several patterns and capacity > 0 (else EINVAL).  On
   ECAPACITY nothing is written to counts_dev and *n_found holds the
   required size.  Errors: as for coex_find. */
int coex_count_find(const coex_dfa* dfa, const coex_seq* seq, uint64_t* counts_dev, int64_t* pos_dev,
                    uint32_t* pattern_dev, uint64_t capacity, uint64_t* n_found, const coex_opts* opts, void* stream);

/* The per-chunk records of Algorithm 1 (CR: init state, last state, counts
   per pattern) for the true starting state of each chunk, for chunks of
   `chunk` bases (the last chunk takes the remainder).  n_chunks =
   ceil(n_bases / chunk) (at least 1).  init_dev/last_dev: uint32[n_chunks];
   counts_dev: uint64[n_chunks * n_patterns].  Asynchronous. */
int coex_count_chunks(const coex_dfa* dfa, const coex_seq* seq, uint32_t chunk, uint32_t* init_dev,
                      uint32_t* last_dev, uint64_t* counts_dev, void* stream);

/* Device consistency failures of unchecked calls, without waiting: enqueues
   on `stream` one kernel that writes to *flags_out (device memory or mapped
   pinned host memory, 4 bytes) the OR of the failure bits kept for the calls
   made so far on `stream` (coex_count, coex_find, coex_count_chunks) and for
   coex_count_noalloc calls on the current device, then clears them.  The
   value is there once the stream reaches the kernel; 0 means every check
   passed, any other value that some call's result is not to be trusted (the
   bits name the check, for diagnosis).  Allocates nothing.  Errors: EINVAL
   (flags_out NULL), EDEVICE. */
int coex_errors_async(void* stream, uint32_t* flags_out);

/* ------------------------------------------------------------ pattern partitioning
   Pattern-based partitioning (Section III.A, Fig. 1b): the patterns split
   into parts, one automaton each, every part scanning the same sequence.  It
   takes k-mer sets whose single automaton would be too large for the device
   tables (more than 4096 states) or for the three-symbol tables (more than
   1023), and gives short inputs more work to run at once. */
typedef struct coex_partition coex_partition;

/* Splits `n` k-mers (as for coex_compile_kmers; pattern id = index) into
   parts whose Aho-Corasick automata have at most `max_states` states (0 =
   1023): patterns in sorted order, a part closed when the next pattern's new
   prefixes would take its trie past the budget.  Errors: EINVAL, EALPHABET,
   ETOOBIG (one k-mer alone needs more states than the budget), ENOMEM. */
int coex_partition_kmers(const char* const* kmers, uint32_t n, uint32_t max_states, coex_partition** out);

int coex_partition_info(const coex_partition* p, uint32_t* n_parts, uint32_t* n_patterns);

/* Part i: its automaton (owned by the partition) and the global ids of its
   patterns (ids[j] = global id of the part's pattern j). */
int coex_partition_part(const coex_partition* p, uint32_t i, const coex_dfa** dfa, const uint32_t** ids,
                        uint32_t* n);

/* Per-pattern counts of every part over `seq` into counts_dev
   uint64[n_patterns] (global ids).  The parts run as coex_count on up to four
   streams of the partition's own, after the work already queued on `stream`;
   the counts are complete, and the parts' consistency failures handed to
   `stream`'s kept word (coex_errors_async), once `stream` passes the call's
   last kernel.  Calls on one partition must not overlap.  Errors: as for
   coex_count. */
int coex_count_partitioned(coex_partition* p, const coex_seq* seq, uint64_t* counts_dev, const coex_opts* opts,
                           void* stream);

void coex_partition_free(coex_partition* p);

/* ------------------------------------------------------------ FASTA ingest
   Host-side parsing of FASTA text (not part of the paper's method: the input
   format of the sequences it scans).  Lines starting with '>' are headers and
   start records; all other lines hold bases; line breaks ("\n", "\r\n") and
   blanks are dropped; bases before the first header form a record of their
   own (a text without headers is one record).  The records are written back
   to back, so the whole output can be scanned at once, or record r alone as
   the n = rec_len[r] bases from first_base = rec_start[r].  Work is split over
   `threads` host threads (0 = every hardware thread) at line starts. */
#define COEX_FASTA_SOFTMASK 1u /* lowercase letters (soft-masked bases) read as N, a reset */
#define COEX_FASTA_SEPARATE 2u /* one N between consecutive records: a whole-output scan never
                                  matches across records */

/* Sizes the output: *n_records, and *n_bases (separators included). */
int coex_fasta_measure(const char* text, uint64_t len, uint32_t flags, uint32_t threads, uint64_t* n_records,
                       uint64_t* n_bases);

/* Parses into host buffers.  COEX_ENC_BYTE: `bases` receives one byte per
   base as written in the text (with COEX_FASTA_SOFTMASK, lowercase letters
   as 'N'; separators are 'N'); n_mask is unused.  COEX_ENC_2BIT: `bases`
   receives ceil(n/4) bytes of codes (A=0 C=1 G=2 T=3, four per byte from the
   low bits) and n_mask, if not NULL, ceil(n/8) bytes whose bit i is set for
   every base i that is not A/C/G/T in either case (and for soft-masked bases
   and separators).  rec_start[r] / rec_len[r]: first base and length of
   record r in the output; rec_header[r]: text offset of its '>' (UINT64_MAX
   for a record before the first header); each may be NULL.  *n_records and
   *n_bases are always set; ECAPACITY (nothing written) when n_bases exceeds
   cap_bases or, with a record array given, n_records exceeds cap_records.
   Errors: EINVAL, ECAPACITY, ENOMEM. */
int coex_fasta_read(const char* text, uint64_t len, int32_t encoding, uint32_t flags, uint32_t threads,
                    void* bases, uint8_t* n_mask, uint64_t cap_bases, uint64_t* rec_start, uint64_t* rec_len,
                    uint64_t* rec_header, uint64_t cap_records, uint64_t* n_records, uint64_t* n_bases);

/* The paper's own method on the host's cores (Section III, Algorithm 1), a
   CPU baseline reported beside the GPU scan (never used by the calls above):
   `n_chunks` equal chunks (0 = one per thread; the last takes the remainder)
   taken by `threads` worker threads (0 = every hardware thread).  Per chunk:
   possible starting states from the symbol before it (Section III.A), the
   first candidate's run R0 over the whole chunk with its state after each of
   the first `window` symbols kept (0 = 4096), every other candidate run
   until it meets R0 after the same number of symbols (the converging point,
   Section III.B.3) or, failing that inside the window, to the chunk end; then
   the join links each chunk's last state to the next chunk's first state and
   the counts are fixed up at the converging point.  Host pointers: bases
   (n_bases bytes, or packed 2-bit codes with the optional n_mask, as
   coex_seq describes), counts uint64[n_patterns].  Synchronous.  Errors:
   EINVAL, ENOMEM, EINTERNAL (the true first state missing from a chunk's
   possible starting states, which the method rules out). */
int coex_count_host(const coex_dfa* dfa, const void* bases, const uint8_t* n_mask, uint64_t n_bases,
                    int32_t encoding, uint32_t threads, uint64_t n_chunks, uint64_t window, uint64_t* counts);

/* ------------------------------------------------------------ batches
   Many sequences and automata in one persistent launch.  Per pair the method
   is the one above (Section III, Algorithm 1): chunks, possible starting
   states from a lookback table, lockstep speculative runs to the converging
   point, one scan of the rest of each chunk, the join and the count fix-up.
   Chunks of one sequence have `chunk` bases except the last, which also takes
   the remainder (a sequence shorter than `chunk` is one chunk). */

typedef struct coex_dfa_set coex_dfa_set;
typedef struct coex_batch coex_batch;

/* Resident automata: their tables packed into LDS groups on the current
   device (two-symbol rows for automata of at most 960 states and at most 15
   patterns per state, one-symbol rows for the others; a group holds up to
   960 or 4096 states of one kind; two-symbol groups also stage their
   one-symbol rows for the speculation).  opts may be NULL; opts->width caps the
   possible starting states of a chunk (1..64, default 64; a lane runs them in
   batches of 8 registers, merging each batch into the next at its converging
   point) and opts->step forces 1 or 2 symbols per lookup.  The set copies
   what it needs from the automata; they may be freed afterwards.  Errors: EINVAL, ETOOBIG (an automaton above 4096
   states), EUNSUPPORTED (an automaton whose possible starting states exceed
   the width at every lookback k <= 8, or more than 255 patterns per state),
   ENOMEM, EDEVICE. */
int coex_dfa_set_create(const coex_dfa* const* dfas, uint32_t n_dfa, const coex_opts* opts, coex_dfa_set** out);
void coex_dfa_set_free(coex_dfa_set* set);

/* A batch over `set`: pairs (pair_seq[i], pair_dfa[i]) of sequence and
   automaton indices, i < n_pairs (host arrays, copied); both NULL = every
   sequence with every automaton, pair index s * n_dfa + d.  Sequences are
   device-resident (16-byte aligned) and must all use one encoding; the batch
   keeps their pointers, so they must stay valid while it is run.
   opts->chunk: bases per chunk (>= 64; 0 = chosen from the batch size and
   the GPU); opts->width: width cap of this batch (a power of two up to the
   set's; 0 = the set's; coex_batch_tune reports the fastest); flags:
   COEX_FLAG_CHECK, COEX_FLAG_TIME (events around the scan
   kernel, or the whole graph; read by coex_batch_info), COEX_FLAG_GRAPH.
   Synchronous (uploads descriptors).  Errors: EINVAL, ENOMEM, EDEVICE. */
int coex_batch_create(const coex_dfa_set* set, const coex_seq* seqs, uint32_t n_seq, const uint32_t* pair_seq,
                      const uint32_t* pair_dfa, uint32_t n_pairs, const coex_opts* opts, coex_batch** out);

/* Points the batch at new sequences and pairs (same rules as
   coex_batch_create), reusing its device buffers when they are large enough.
   The batch must not be running.  Synchronous (uploads descriptors). */
int coex_batch_update(coex_batch* batch, const coex_seq* seqs, uint32_t n_seq, const uint32_t* pair_seq,
                      const uint32_t* pair_dfa, uint32_t n_pairs);

/* Runs the batch: counts_dev uint64[n_pairs] receives the total number of
   matches (all pattern ids) of each pair.  Asynchronous on `stream` unless
   COEX_FLAG_CHECK was given.  Runs of one batch must not overlap. */
int coex_batch_run(coex_batch* batch, uint64_t* counts_dev, void* stream);

/* Autotuner: runs the batch for every speculation width cap 1, 2, 4, ...
   up to the set's (opts->width at coex_dfa_set_create, default 64; the cap
   picks each automaton's lookback, and so how many possible starting states
   its chunks speculate on; caps that pick the same lookbacks for every
   automaton run once) crossed with chunk lengths 4 KiB, 16 KiB, ..., 1 MiB,
   times each with HIP events (after one warm-up run each), keeps the
   fastest pair and reports it in *chunk_out and *width_out (may be NULL).
   counts_dev as for coex_batch_run (holds the last run's exact counts).
   Synchronises `stream`. */
int coex_batch_tune(coex_batch* batch, uint64_t* counts_dev, void* stream, uint64_t* chunk_out,
                    uint32_t* width_out);

typedef struct {
  uint64_t chunk;     /* bases per chunk */
  uint32_t width;     /* largest possible-starting-state list of any automaton under the batch's
                         width cap (the set's, or the tuner's choice) */
  uint32_t step;      /* symbols per LDS lookup: 1 or 2 (every group), 3 = groups of both kinds */
  uint32_t n_groups;  /* LDS groups of the automaton set */
  uint32_t n_pairs;
  uint32_t n_tasks;   /* 768-lane tasks of the persistent launch */
  uint32_t blocks;    /* persistent blocks */
  uint64_t n_lanes;   /* (chunk, automaton) work items */
  double last_ms;     /* device time of the last COEX_FLAG_TIME run, -1 if none (waits for it) */
} coex_batch_info_t;

int coex_batch_info(const coex_batch* batch, coex_batch_info_t* info);
void coex_batch_free(coex_batch* batch);

/* Convenience: counts_dev[s * n_dfa + d] = total number of matches of
   dfas[d] in seqs[s] (set + batch + one run, then both freed).  Synchronises
   `stream`. */
int coex_count_batched(const coex_dfa* const* dfas, uint32_t n_dfa, const coex_seq* seqs, uint32_t n_seq,
                       uint64_t* counts_dev, const coex_opts* opts, void* stream);

/* ------------------------------------------------------------ serving
   A serving loop over resident automata: requests (one host sequence of
   ASCII bases and one automaton index each) are admitted in arrival order
   into a device arena of `hbm_budget` bytes, copied on a copy stream while
   earlier batches run (in pieces of `copy_piece` bytes, the request with the
   fewest bytes left first), and every admitted request whose copy has
   finished is launched in the next batch (continuous batching; up to two
   batches in flight, each on a compute stream of its own, so one can run
   while the other is being launched or drained).  A request's count is its
   pair's count in a batch,
   so it is the same alone or in any mix.  One worker thread per server;
   submit and wait may be called from any thread. */

typedef struct coex_server coex_server;

typedef struct {
  uint64_t hbm_budget;  /* bytes of device memory for admitted sequences (0 = 4 GiB) */
  uint32_t max_batch;   /* requests per launch (0 = 1024) */
  uint32_t chunk;       /* bases per chunk (0 = chosen per batch) */
  uint32_t width;       /* as coex_dfa_set_create */
  uint32_t flags;       /* reserved, 0 */
  uint64_t copy_piece;  /* bytes per host-to-device copy piece (0 = 16 MiB); at most three
                           pieces' worth of bytes is queued on the copy stream at a time */
} coex_server_opts;

typedef struct {
  double queue_ms;          /* submit -> admitted (arena space granted) */
  double h2d_ms;            /* device time from the start of the request's first copy piece to the
                               end of its last (other requests' pieces may run in between) */
  double device_ms;         /* device time of the request's batch (launch to counts copied back) */
  double total_ms;          /* submit -> result available on the host */
  double launch_to_done_ms; /* batch launch -> result available (host clock) */
  uint32_t batch_size;      /* requests in the request's batch */
} coex_request_stats_t;

typedef struct {
  uint64_t n_submitted, n_done, n_batches, bases_done;
  uint64_t arena_bytes, max_arena_bytes;
  double device_ms;         /* summed device time of finished batches */
} coex_server_stats_t;

/* Creates a server on the current device over a copy of the automata (the
   handles may be freed afterwards) and starts its worker thread.  opts may be
   NULL.  Errors: as coex_dfa_set_create, ENOMEM for the arena. */
int coex_server_create(const coex_dfa* const* dfas, uint32_t n_dfa, const coex_server_opts* opts,
                       coex_server** out);

/* Queues one request.  host_bases (n_bases ASCII bytes) must stay valid and
   unchanged until coex_server_wait returns for the ticket; page-locked
   memory lets its copy overlap running batches.  Never blocks on the GPU.
   Errors: EINVAL (bad automaton index or NULL pointer). */
int coex_server_submit(coex_server* server, const void* host_bases, uint64_t n_bases, uint32_t dfa,
                       uint64_t* ticket);

/* Blocks until the request is done; *count receives its number of matches
   (all pattern ids) and *stats (may be NULL) its latencies.  Each ticket is
   waited for once.  Returns the request's status (ENOMEM if it can never fit
   the arena, EDEVICE on a runtime error). */
int coex_server_wait(coex_server* server, uint64_t ticket, uint64_t* count, coex_request_stats_t* stats);

int coex_server_stats(coex_server* server, coex_server_stats_t* stats);

/* Finishes every queued request, stops the worker and frees the server. */
void coex_server_free(coex_server* server);

const char* coex_strerror(int status);

/* Instrumentation, not part of the method: total device time (ms) of the
   scan kernel over the calls made on `stream` with COEX_FLAG_TIME since the
   last reset, measured with HIP events recorded on that stream around the
   kernel launch, and the number of such launches.  Waits for those events.
   reset != 0 starts a new measurement window (at most 4096 launches are
   recorded per window). */
int coex_profile(void* stream, double* total_ms, uint64_t* launches, int reset);

/* Version string of the library build. */
const char* coex_version(void);

#ifdef __cplusplus
}
#endif
#endif /* COEX_H */
