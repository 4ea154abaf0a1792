/*
 * slpf.h -- C ABI of the MI355X (gfx950) chunk-parallel RE parser.
 *
 * The library implements the parallel parser of "A parallel parser for
 * regular expressions" (Borsotti, Breveglieri, Crespi Reghizzi, Morzenti,
 * arXiv 2503.06763).  The paper states the problem as two steps: generate
 * the parser automaton of an RE, then parse a text into the shared
 * linearized parse forest (SLPF) of all its syntax trees (Sect. 2.1, "What is
 * RE parsing"; Sect. 4.1, tool structure).  The two calls below follow that
 * split: slpf_compile() on the host, slpf_parse() on the GPU.
 *
 * Conventions for every entry point:
 *  - No exceptions cross the ABI; every call returns an slpf_status
 *    (negative on failure) unless stated otherwise.
 *  - "_dev" pointers are device (HIP global memory) pointers owned by the
 *    caller; the library never frees them.
 *  - Host pointers are only read during the call.
 *  - Calls taking a hip_stream (a hipStream_t, NULL = the default stream)
 *    are asynchronous and stream-ordered: results are valid once the stream
 *    reaches the point of the call (slpf_get_matches and slpf_tune return
 *    after synchronizing the stream).
 *  - A compiled parser is immutable and may be used concurrently from
 *    several host threads and streams.
 *
 * RE syntax: bytes are terminals; metacharacters ( ) | * + ?; a backslash
 * makes the next byte a terminal, with \n, \t and \xHH as shorthands; "()"
 * and an empty alternative denote the empty string epsilon (App. A, "Empty
 * string").  Iterators bind tighter than concatenation, concatenation
 * tighter than union (Sect. 2.1).  A chain of the same operator written
 * without parentheses is one n-ary node; a parenthesised operator
 * subexpression is a node of its own (App. A, "Extra parenthesis").  e? is
 * optionality, numbered like any operator (App. A, "Bounded repetition").
 */
#ifndef SLPF_H
#define SLPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLPF_OK = 0,
    SLPF_E_ARG = -1,        /* bad argument (NULL pointer, bad struct_size, misaligned text) */
    SLPF_E_SYNTAX = -2,     /* RE syntax error; *err_offset = byte offset */
    SLPF_E_INF_AMBIG = -3,  /* an iterator over a nullable body (App. A, "Infinite ambiguity") */
    SLPF_E_TOO_LARGE = -4,  /* automaton beyond the limits (segments, states, entry lists) */
    SLPF_E_NOMEM = -5,      /* host or device allocation failed */
    SLPF_E_DEVICE = -6,     /* a HIP call failed */
    SLPF_E_CAPACITY = -7,   /* output too small: slpf_forest_bytes(), slpf_compact_bytes(), match pairs */
    SLPF_E_INTERNAL = -8
} slpf_status;

typedef struct slpf_parser slpf_parser;   /* opaque, immutable after compile */

/* ------------------------------------------------------------------ compile */

enum {
    SLPF_COMPILE_HOST_ONLY = 1u << 0   /* keep the tables on the host: inspection only, no parse */
};

typedef struct {
    uint32_t struct_size;    /* sizeof(slpf_compile_opts) */
    uint32_t flags;          /* SLPF_COMPILE_* */
    uint32_t max_segments;   /* 0 = default and maximum: 2048 (32 words per column) */
    uint32_t max_states;     /* per direction, 0 = default (65535, the u16 id range) */
    int32_t device;          /* HIP device ordinal that will run the parses */
} slpf_compile_opts;

/*
 * Compile an RE into its parser automaton (Sect. 2.2-3.1): number the RE,
 * compute the classic followers, the segments (Fig. segmentalgo), the
 * follower segments (Eq. folsegdef), and by powerset the forward and reverse
 * tables.  Each direction's table is the union of the DFA started from the
 * initial (resp. final) set and the multi-entry DFA started from every
 * singleton segment, identical segment sets merged (Sect. 3.1 and the
 * "Automaton optimization" paragraph of Sect. 3.3); the DFA is never
 * minimized (Sect. 3.1).  The tables are uploaded to `device`.
 *
 * re/re_len: the RE bytes (not NUL-terminated; may contain NUL).
 * opts: may be NULL for defaults.  With SLPF_COMPILE_HOST_ONLY nothing is
 *   uploaded and no HIP call is made (a parse with such a parser returns
 *   SLPF_E_ARG); the inspection calls below work as usual.
 * out: receives the parser; *out = NULL on failure.
 * err_offset: may be NULL; set to the failing byte offset on SLPF_E_SYNTAX.
 */
slpf_status slpf_compile(const char *re, size_t re_len, const slpf_compile_opts *opts,
                         slpf_parser **out, size_t *err_offset);

/* Free a parser and its device tables.  The caller must ensure no parse
 * using it is still running on any stream.  NULL is ignored. */
void slpf_parser_destroy(slpf_parser *p);

typedef struct {
    uint32_t num_segments;       /* l = |Q|, states of the parser NFA */
    uint32_t words_per_column;   /* W = ceil(l / 64) */
    uint32_t num_initial, num_final;
    uint32_t fwd_states;         /* forward table, the empty set excluded */
    uint32_t rev_states;         /* reverse table, the empty set excluded */
    uint32_t dfa_states;         /* forward DFA from I (Sect. 3.2 "DFA") */
    uint32_t medfa_states;       /* forward ME-DFA from the singletons */
    uint32_t rdfa_states;        /* reverse DFA from F */
    uint32_t rmedfa_states;      /* reverse ME-DFA from the singletons */
    uint32_t num_classes;        /* byte classes, class 0 = bytes outside the RE */
    uint32_t max_entries;        /* longest speculative entry list (join masks take
                                    ceil(max_entries / 64) words) */
    uint32_t placement;          /* 0 = transition tables staged in LDS, 1 = read through L2 */
    uint32_t max_entries_next_byte;  /* longest entry list without the previous-byte filter
                                        (the lists of SLPF_PARSE_NEXT_BYTE_ENTRIES) */
    uint32_t column_unambiguous; /* 1 when no forward state reachable from I and reverse state
                                    reachable from F share two segments: every clean column of an
                                    accepted text is then one segment and the text has one tree */
    uint32_t reserved;
    uint64_t table_bytes;        /* device bytes of all tables */
} slpf_parser_info;

slpf_status slpf_parser_info_get(const slpf_parser *p, slpf_parser_info *info);

/*
 * Text of segment `seg` (0-based, canonical order: by end-letter number with
 * the end mark last, then meta-prefix length, then the meta-prefix symbols
 * compared as (number, kind) with "(" < leaf < ")").  Symbols are separated
 * by one space: "k(" and ")k" for the numbered parentheses of operator k, a
 * terminal as its letter followed by its number ("a4"; bytes other than
 * ASCII letters as "\xHH" then the number), "ε" + number for an epsilon
 * leaf, "⊣" (UTF-8) for the end mark.  Writes at most cap bytes including
 * a terminating NUL; *need (may be NULL) receives the length without NUL.
 */
slpf_status slpf_segment_text(const slpf_parser *p, uint32_t seg, char *buf, size_t cap,
                              size_t *need);

/*
 * Host copy of one direction's merged table (dir 0 forward, 1 reverse):
 * sets: (states+1) x W words, row 0 the empty set; delta: (states+1) x
 * num_classes ids; classmap: 256 class ids.  Any pointer may be NULL.
 * Sizes come from slpf_parser_info_get.
 */
slpf_status slpf_table_dump(const slpf_parser *p, int dir, uint64_t *sets, uint32_t *delta,
                            uint16_t *classmap);

/* Bytes of the SLPF of an n-byte text: (n + 1) * W * 8. */
uint64_t slpf_forest_bytes(const slpf_parser *p, uint64_t n);

/*
 * Compact SLPF (App. SLPF optimization, SLPF encoding).  Every segment of
 * the clean column C_r follows a segment labelled x_r and has the end-letter
 * x_{r+1}, so C_r lies in the candidate list X(x_r, x_{r+1}): the segments
 * with end-letter class of x_{r+1} (final segments at r = n) that follow a
 * segment labelled with the class of x_r (initial segments at r = 0),
 * ascending by segment id.  When every such list holds at most 64 segments
 * (slpf_parser_info.max_entries <= 64), the compact column r is one
 * uint64_t whose bit k is set iff the k-th segment of X(x_r, x_{r+1}) is in
 * C_r: (n + 1) * 8 bytes for the whole SLPF instead of (n + 1) * W * 8.
 * Parsers with longer lists have no compact form: SLPF_PARSE_COMPACT and
 * slpf_decode_compact return SLPF_E_TOO_LARGE for them.
 */
uint64_t slpf_compact_bytes(uint64_t n);

/*
 * Expand a compact SLPF (compact_dev, n + 1 words, from a parse of text_dev
 * with SLPF_PARSE_COMPACT) into the W-word columns of slpf_forest
 * (columns_dev, slpf_forest_bytes(p, n) bytes).  Device pointers; the text
 * gives each column's candidate list.  Stream-ordered on hip_stream.
 * SLPF_E_ARG on a NULL pointer (text_dev may be NULL when n = 0).
 */
slpf_status slpf_decode_compact(const slpf_parser *p, const uint8_t *text_dev, uint64_t n,
                                const uint64_t *compact_dev, uint64_t *columns_dev, void *hip_stream);

/*
 * Match extraction (Sect. 4, Other functions of the tool: getMatches).  The
 * matches of group `group` -- the operator node with that number in the
 * preorder numbering of the RE, as printed by slpf_segment_text ("g(" and
 * ")g") -- in the clean SLPF columns_dev of an n-byte text (the W-word
 * layout of slpf_parse, device memory): every pair (start, end) of text
 * positions, 0 <= start <= end <= n, such that some syntax tree of the text
 * has "g(" at position start and its matching ")g" at position end, i.e. the
 * group's substring is text[start, end).  A rejected text has none.
 *
 * pairs_dev: device, room for `capacity` pairs of uint64_t (start, end),
 *   written sorted by (start, end).
 * *num_matches (host): the number of matches.  SLPF_E_CAPACITY when it
 *   exceeds capacity (the first `capacity` pairs are written).
 * SLPF_E_ARG: NULL pointer, group 0 or past the last node number, n >= 2^31 - 1.
 * Work buffers are allocated for the call; the call synchronizes hip_stream.
 * The cost is proportional to the summed lengths of the matches.
 */
slpf_status slpf_get_matches(const slpf_parser *p, const uint64_t *columns_dev, uint64_t n, uint32_t group,
                             uint64_t *pairs_dev, uint64_t capacity, uint64_t *num_matches, void *hip_stream);

/*
 * Child extraction (Sect. 4, Other functions of the tool: getChildren).
 * Given a match (start, end) of node `group` (as slpf_get_matches lists
 * them) in the clean SLPF columns_dev of an n-byte text, the matches of its
 * children: every triple (k, a, b) such that some syntax tree of the text
 * holds `group` over text[start, end) and, directly inside that occurrence,
 * node k over text[a, b).  k is a child of `group` in the RE tree (an
 * operand of a concatenation or union, the body of a star, cross or
 * optional part); a terminal child spans one byte (b = a + 1), an epsilon
 * child or an empty operator child none (b = a).  A pair (start, end) that
 * is no match of the node, and a leaf node, have no children.
 *
 * triples_dev: device, room for `capacity` triples of uint64_t (k, a, b),
 *   written sorted by (k, a, b).
 * *num_children (host): the number of triples.  SLPF_E_CAPACITY when it
 *   exceeds capacity (the first `capacity` triples are written).
 * SLPF_E_ARG: NULL pointer, group 0 or past the last node number,
 *   start > end, end > n, n >= 2^31 - 1, or (number of children of the node)
 *   x (end - start + 1) >= 2^31 - 1.
 * Work buffers are allocated for the call (about (8 W + 25 k + 9) bytes per
 * column of the span, k the node's number of children); the call
 * synchronizes hip_stream.  The columns of the span are cut into stretches at
 * the columns that hold one segment; the cost is proportional to the span's
 * length plus the summed lengths of the child matches, and the longest
 * stretch of columns with several segments runs in one wavefront.
 */
slpf_status slpf_get_children(const slpf_parser *p, const uint64_t *columns_dev, uint64_t n, uint32_t group,
                              uint64_t start, uint64_t end, uint64_t *triples_dev, uint64_t capacity,
                              uint64_t *num_children, void *hip_stream);

/* -------------------------------------------------------------------- parse */

enum {
    SLPF_PARSE_NO_COUNT = 1u << 0,      /* skip the tree count (scalars[1] = [3] = 0, [2] = 2) */
    SLPF_PARSE_FORCE_L2 = 1u << 1,      /* read transition tables through L2 even if LDS fits */
    SLPF_PARSE_RECOGNIZE = 1u << 2,     /* recogniser only (Sect. 3.2: the forward reacher and joiner
                                           decide membership): scalars[0] = accept, [1] = [3] = 0,
                                           [2] = 2;
                                           no column is written (columns_dev may be NULL) */
    SLPF_PARSE_COMPACT = 1u << 3,       /* write the compact SLPF (App. SLPF optimization, SLPF
                                           encoding): column r as ONE word; see slpf_decode_compact.
                                           capacity_bytes >= slpf_compact_bytes(n) */
    SLPF_PARSE_NEXT_BYTE_ENTRIES = 1u << 4, /* speculation ablation: each lane chunk's runs start
                                           from every segment whose end-letter is the chunk's first
                                           byte (the ME-DFA entries of Sect. 3.1 for that letter),
                                           without the filter by the previous byte.  Same results */
    SLPF_PARSE_EDGE_SHIFT = 1u << 5,    /* chunk-edge shifting on (Sect. Tool optimization, technique
                                           (ii)): the speculative runs and the join of a lane chunk
                                           start at the position, within a window after its edge,
                                           whose entry list is shortest.  Same results.  Default: on
                                           when the parser's entry lists exceed 12 segments */
    SLPF_PARSE_NO_EDGE_SHIFT = 1u << 6, /* chunk-edge shifting off (wins over SLPF_PARSE_EDGE_SHIFT) */
    SLPF_PARSE_ALL_DFA_STATES = 1u << 7, /* speculation ablation, the standard scheme the ME-DFA entries
                                           are compared with (Sect. 5): a lane chunk's runs start from
                                           every state of the forward (reverse) DFA at its inner edges,
                                           from I (F) at the text's first (last) edge.  Same results;
                                           no chunk-edge shifting.  SLPF_E_TOO_LARGE when a DFA has
                                           more than 2048 states */
    SLPF_PARSE_WIDE_COUNT = 1u << 8     /* tree count: the short runs of ambiguous columns are counted
                                           with 16-segment vectors at once, without the 8-segment pass
                                           first; faster when most of them hold columns of more than 8
                                           segments, identical results.  slpf_tune tries it. */
};

typedef struct {
    uint32_t struct_size;     /* sizeof(slpf_parse_opts) */
    uint32_t chunk_bytes;     /* bytes per lane chunk, a multiple of 64; 0 = automatic */
    uint32_t flags;           /* SLPF_PARSE_* */
    uint32_t reserved;
    uint64_t *trace_dev;      /* optional: receives the join results, see below */
    uint64_t trace_bytes;     /* capacity of trace_dev */
    void *const *events;      /* optional: SLPF_NUM_PHASE_EVENTS caller-created hipEvent_t */
    uint32_t num_events;      /* 0, or SLPF_NUM_PHASE_EVENTS */
    uint32_t reserved2;
} slpf_parse_opts;

/* Phase events: when opts->events is set, events[k] is recorded on the parse
 * stream before reach (0), after reach (1), after the join scans (2), after
 * the join start ids (3), after build & merge (4) and after the tree count
 * (5), so that hipEventElapsedTime gives each phase's device time. */
#define SLPF_NUM_PHASE_EVENTS 6

/*
 * Output of a parse.  columns_dev: the SLPF, column r (0 <= r <= n) at
 * words [r*W, (r+1)*W), bit j of the column set iff segment j is in the
 * clean column C_r (Sect. 2.3.4; Boolean vectors as in Sect. 2.4); with
 * SLPF_PARSE_COMPACT, word r is the compact column (see slpf_compact_bytes).
 * scalars_dev[0] = 1 if the text is in the language else 0;
 * scalars_dev[1] = number of syntax trees modulo 2^64 (the number of
 *                  accepting NFA runs, one per LST, Sect. 2.3.4);
 * scalars_dev[2] = 0 if scalars_dev[1] and [3] are valid, 1 if the count
 *                  was not computed (a run of ambiguous columns with a column
 *                  of more than 1024 segments, or a run longer than 512
 *                  columns cut into pieces where a column after its first
 *                  piece holds more than 128 segments), 2 if not requested
 *                  (SLPF_PARSE_NO_COUNT), 3 on an internal error (a join set
 *                  missing from the tables);
 * scalars_dev[3] = number of syntax trees modulo the prime 2^61 - 1 (a
 *                  second check that does not vanish when the count is a
 *                  multiple of 2^64).
 * The count is the same for every lane-chunk size and with batching.
 * columns_dev must be 8-byte aligned; with 128-byte alignment every store
 * of the build covers whole cache lines.
 */
typedef struct {
    uint64_t *columns_dev;     /* device, capacity_bytes >= slpf_forest_bytes(p, n), or
                                  slpf_compact_bytes(n) with SLPF_PARSE_COMPACT */
    uint64_t capacity_bytes;
    uint64_t *scalars_dev;     /* device, 4 words */
} slpf_forest;

/*
 * Parse text_dev[0..n) into its clean SLPF (Sect. 3.2-3.3): split into lane
 * chunks, speculative forward and backward reach from the reduced entry
 * sets (Eq. reacher), join of the chunk maps (Eq. joiner), fused build and
 * merge (Eq. builder, Eq. merger, Fig. builders&merger), composition of
 * column 0, and the tree count.
 *
 * text_dev: device pointer, 16-byte aligned, n readable bytes.  Bytes
 *   outside the RE's alphabet are not errors: the text is rejected, every
 *   column is empty and the count is 0.
 * opts: may be NULL for defaults.  If opts->trace_dev is set and
 *   trace_bytes >= 2 * (c + 1) * W * 8 (c = number of lane chunks,
 *   ceil(n / chunk_bytes)), the forward join sets J (the forward column at
 *   every lane-chunk edge) and then the backward sets J^ (the backward
 *   column at every edge) are written there, (c + 1) x W words each.
 * forest: output buffers; SLPF_E_CAPACITY if too small.
 * hip_stream: hipStream_t or NULL.
 * Work buffers are allocated by the library and kept with the parser; a
 * parse that needs a larger workspace than a previous one synchronizes the
 * stream before reallocating.
 */
slpf_status slpf_parse(const slpf_parser *p, const uint8_t *text_dev, uint64_t n,
                       const slpf_parse_opts *opts, const slpf_forest *forest, void *hip_stream);

/*
 * slpf_parse for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, and harnesses that forbid hipMalloc.  Same
 * arguments, results and stream order as slpf_parse, but the work buffers
 * come from a library-owned device array of 128 MiB (one per GPU, held until
 * the process ends) instead of a per-stream allocation; no hipMalloc,
 * hipFree or other allocating call is made (the array's device address is
 * looked up once per device on the first call there).  The clearing the
 * parse needs is done by its own first kernel.
 *
 * SLPF_E_CAPACITY when the parse's work buffers would exceed the 128 MiB
 * array: with entry lists of up to 64 segments they take about
 * (38 E + 60) / s + 2.4 bytes per text byte (E = slpf_parser_info.max_entries,
 * s = lane-chunk bytes), so the 304-segment random RE of the single-RE
 * workload (E = 10) fits texts of 24 MiB with the automatic chunking
 * (256-byte lane chunks at that size); other errors as for
 * slpf_parse.  Every call on one GPU uses the
 * same array and leaves its last contents there: calls that overlap on one
 * GPU (on different streams, or from several threads) race and must be
 * serialized by the caller.
 */
slpf_status slpf_parse_noalloc(const slpf_parser *p, const uint8_t *text_dev, uint64_t n,
                               const slpf_parse_opts *opts, const slpf_forest *forest, void *hip_stream);

/* One text of a batch: its device bytes and its output buffers (as for
 * slpf_parse; each text needs its own columns and scalars). */
typedef struct {
    const uint8_t *text_dev;
    uint64_t n;
    slpf_forest out;
} slpf_text;

/*
 * Parse `count` texts with one parser in one job (the batched form of
 * slpf_parse).  The lane chunks of all texts form one index space, so one
 * launch of each phase covers every text and thousands of small texts fill
 * the GPU; the join is a scan segmented at text boundaries.  Results are
 * identical to parsing each text alone.  Every item must satisfy the
 * conditions of slpf_parse (alignment, capacity); the first violation is
 * returned and nothing is launched.  opts->chunk_bytes applies to every
 * text; the join trace is not available for batches.  The descriptors are
 * copied from a pinned staging buffer on the stream; the host waits for the
 * previous batch's copy on the same stream before reusing that buffer.
 */
slpf_status slpf_parse_texts(const slpf_parser *p, const slpf_text *items, size_t count,
                             const slpf_parse_opts *opts, void *hip_stream);

/* One text of a batch over many parsers: its parser, device bytes and
 * output buffers (as for slpf_parse). */
typedef struct {
    const slpf_parser *p;
    const uint8_t *text_dev;
    uint64_t n;
    slpf_forest out;
} slpf_item;

/*
 * Parse `count` texts, each with its own parser, in one call: the batched
 * form over many REs.  The items of one parser form one job (as
 * slpf_parse_texts); the jobs of different parsers run concurrently on
 * library-owned streams of the device (a few per GPU, forked from and joined
 * back into hip_stream, so the call is ordered on hip_stream like any other
 * launch).  Results are identical to parsing each text alone.  Every parser
 * must live on the device of hip_stream, and every item must satisfy the
 * conditions of slpf_parse; the first violation is returned and nothing is
 * launched.  With opts->chunk_bytes = 0 a parser that slpf_tune has tuned
 * uses its tuned lane-chunk size, table placement and count width.  A failure of one job
 * (e.g. SLPF_E_NOMEM) is returned after the jobs already launched have been
 * joined into hip_stream.  Calls that overlap on one device are serialized
 * by the library.
 */
slpf_status slpf_parse_batch(const slpf_item *items, size_t count, const slpf_parse_opts *opts,
                             void *hip_stream);

/*
 * Free the work buffers the parser keeps for parses on hip_stream (after
 * synchronizing that stream); call before destroying a stream the parser was
 * used on.  Later parses on the stream allocate them again.
 */
slpf_status slpf_parser_trim(const slpf_parser *p, void *hip_stream);

/*
 * Autotuner: time one batched parse of `items` (slpf_parse_texts, after one
 * untimed run) for
 * every lane-chunk size in {256, 512, 1024, 2048, 4096} bytes and, when the
 * tables fit in LDS, both table placements (LDS and L2), and, when the trees
 * are counted in runs, both count widths (with and without
 * SLPF_PARSE_WIDE_COUNT), and return the fastest in best->chunk_bytes and
 * best->flags (`flags` plus SLPF_PARSE_FORCE_L2 and SLPF_PARSE_WIDE_COUNT
 * when they won; both are ignored in `flags`); *best_ms (may be NULL)
 * receives its time.  best->struct_size must be set; its other fields are
 * overwritten.  The items' outputs hold a complete parse on return (every
 * candidate computes the same result).  The parser keeps the result for
 * slpf_parse_batch.  Synchronizes the stream.
 */
slpf_status slpf_tune(const slpf_parser *p, const slpf_text *items, size_t count, uint32_t flags,
                      slpf_parse_opts *best, float *best_ms, void *hip_stream);

/* ---------------------------------------------------------------- server
 *
 * Continuous batching of parse requests on one GPU (for serving): parsers
 * stay resident, requests queue in FIFO order, and a request is admitted
 * when a job slot is free and the SLPF it will produce (slpf_forest_bytes,
 * plus the scalars) fits in the server's device arena of memory_budget
 * bytes.  The requests admitted into a slot run as one job (per parser, one
 * slpf_parse_texts) on that slot's stream; slots run concurrently.  Results
 * are identical to slpf_parse of each text alone (see slpf_parse_texts for
 * the one exception).  A server is driven from one host thread.
 */
typedef struct slpf_server slpf_server;

typedef struct {
    uint32_t struct_size;        /* sizeof(slpf_server_opts) */
    uint32_t slots;              /* jobs in flight at once (each on its own stream) */
    uint32_t max_batch_texts;    /* requests admitted into one job at most */
    uint32_t parse_flags;        /* SLPF_PARSE_* for every job */
    uint64_t memory_budget;      /* bytes of the output arena (allocated at create) */
    int32_t device;
    uint32_t reserved;
} slpf_server_opts;

typedef struct {
    uint64_t queued, in_flight, busy_slots, finished_unreleased;
    uint64_t admitted_bytes, arena_bytes;
} slpf_server_state;

slpf_status slpf_server_create(const slpf_server_opts *opts, slpf_server **out);
/* Waits for the jobs in flight, then frees the arena, the streams and the
 * work buffers the parsers kept for those streams.  Parsers used by the
 * server must outlive it. */
void slpf_server_destroy(slpf_server *s);
/* Queue a request: text_dev (16-byte aligned, n bytes) stays owned by the
 * caller and must stay valid until the request is reported done; its bytes
 * must already be in place (the server's streams do not wait for work on
 * other streams).  tag
 * identifies the request in slpf_server_poll/result/release and must be
 * unique among requests not yet released.  SLPF_E_CAPACITY if its output
 * alone exceeds the budget. */
slpf_status slpf_server_submit(slpf_server *s, const slpf_parser *p, const uint8_t *text_dev, uint64_t n,
                               uint64_t tag);
/* Retire finished jobs, admit and launch queued requests into free slots,
 * and report up to cap finished tags (the rest are reported by later
 * calls).  Does not block on the GPU. */
slpf_status slpf_server_poll(slpf_server *s, uint64_t *done_tags, size_t cap, size_t *n_done);
/* Output of a finished request (device pointers into the arena, valid until
 * slpf_server_release).  Returns the request's parse status: a request whose
 * job could not be launched (slpf_parse_texts failed for its parser, e.g. a
 * parser compiled with SLPF_COMPILE_HOST_ONLY) is still reported finished by
 * slpf_server_poll, and this call then returns that error; the requests of
 * the other parsers in the same slot are not affected. */
slpf_status slpf_server_result(const slpf_server *s, uint64_t tag, slpf_forest *out);
/* Return a finished request's arena space. */
slpf_status slpf_server_release(slpf_server *s, uint64_t tag);
slpf_status slpf_server_stats(const slpf_server *s, slpf_server_state *state);

/* Number of lane chunks a parse of n bytes uses with the given options. */
uint64_t slpf_num_chunks(const slpf_parser *p, uint64_t n, const slpf_parse_opts *opts);

const char *slpf_status_str(slpf_status s);

#ifdef __cplusplus
}
#endif

#endif /* SLPF_H */
