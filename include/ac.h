/*
 * ac.h -- C ABI of the MI355X (gfx950) Aho-Corasick scan library, libac.so.
 *
 * The library finds every occurrence of a set of byte patterns in a byte
 * text, the multiple-string-matching problem of the paper (abstract, Sec. I).
 * It does so the way the paper's Sec. II splits the method: a host step that
 * constructs the string-matching machine (ac_build), and a device step that
 * processes the text with it in one pass (ac_scan).
 *
 * Result convention (shared by every scan entry point):
 *   a match is the 64-bit key (e << 32) | k, meaning pattern k (its 0-based
 *   index in the list given to ac_build) ends at 0-based text position e.
 *   Every occurrence is reported, including overlapping ones and patterns
 *   nested inside others (the Sec. IV.A example reports both SHE and HE).
 *   Duplicate patterns each report their own id. Keys are written in an
 *   unspecified order; sorted ascending they give the list ordered by
 *   (e, k). Texts must be shorter than 2^32 bytes.
 *
 * Memory: texts, match buffers and counters passed to scans are device
 * pointers owned by the caller. The automaton owns its host and device
 * tables until ac_free. Streams are hipStream_t values passed as void*;
 * NULL means the default stream. Calls never throw; they return AC_OK or a
 * negative AC_ERR_* code and leave a message for ac_last_error().
 */
#ifndef AC_H
#define AC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    AC_OK = 0,
    AC_ERR_INVALID = -1,   /* bad argument: null pointer, empty pattern, misaligned text */
    AC_ERR_NOMEM = -2,     /* host or device allocation failed */
    AC_ERR_TOO_LARGE = -3, /* machine or text beyond the index ranges below */
    AC_ERR_OVERFLOW = -4,  /* more matches than the buffer holds (ac_scan_sync) */
    AC_ERR_HIP = -5,       /* a HIP runtime call failed */
    AC_ERR_BUSY = -6       /* resource budget exhausted (serving) */
};

/* Where the transition table lives during a scan. */
enum {
    AC_PLACE_AUTO = 0,   /* LDS_FULL if the table fits a workgroup's LDS, else LDS_HOT */
    AC_PLACE_GLOBAL = 1, /* every lookup from global memory (L2 / MALL resident) */
    AC_PLACE_LDS_FULL = 2, /* the whole 32-bit table copied into LDS */
    AC_PLACE_LDS_HOT = 3   /* 16-bit rows of the most visited states in LDS, rest global */
};

/* Which device matcher a scan runs. Every one reports the same matches. */
enum {
    AC_ALGO_AUTO = 0,  /* GATED when the automaton has a start-position gate that
                          is expected to pass at most 1 start position in 20,
                          else DFA (PFAC for a goto-only automaton) */
    AC_ALGO_DFA = 1,   /* failure transitions folded into a full DFA, walked over
                          overlapping chunks of the text */
    AC_ALGO_PFAC = 2,  /* failure-less machine, one walk per start position */
    AC_ALGO_GATED = 3  /* failure-less machine, walked only from the start
                          positions whose next bytes can begin a pattern, as
                          a bitmap held in LDS decides. The class gate (patterns
                          over at most four letters told apart by a 2-bit field
                          of the byte) covers the 4^10 class strings of 10
                          bytes, and a table over them takes the walk's first
                          10 steps at once. The hashed gate (every pattern 6
                          bytes or longer) is a blocked Bloom filter over the
                          patterns' first 6 bytes, and a hash table of those
                          windows takes the first 6 steps (ac_info_t.has_gate,
                          gate_pass) */
};

typedef struct ac_automaton ac_automaton;

typedef struct {
    uint32_t placement;   /* AC_PLACE_*; default AC_PLACE_AUTO */
    uint32_t hot_states;  /* cap on states in the LDS_HOT image; 0 = as many as fit */
    uint32_t lds_bytes;   /* LDS budget for the table image; 0 = 151 KiB (the rest of
                             the 160 KiB holds per-wave match queues) */
    uint32_t flags;       /* AC_BUILD_* bits */
    uint32_t threads;     /* host threads for the construction (level by level in
                             breadth-first order; the result does not depend on it);
                             0 = hardware threads, at most 16 */
    uint32_t reserved;
} ac_build_opts;

enum {
    /* Failure-less machine only (Sec. II.B): the goto function and the
     * patterns ending at each state, without failure function, output unions
     * or full DFA. Cheaper to build (Sec. IV.A, the cost the paper reduces);
     * such an automaton scans with AC_ALGO_PFAC or AC_ALGO_GATED only. */
    AC_BUILD_GOTO_ONLY = 1,
    /* Also build two-byte rows for the states outside the LDS_HOT image
     * (4-column hashed machines with an image and at most 2^20 such states):
     * a DFA scan then looks up two bytes at once from those states. Halves
     * the dependent global lookups, but the rows are 16 times the one-byte
     * rows and miss L2 more often, so it is off by default. */
    AC_BUILD_PAIR_ROWS = 2,
    /* Do not build the start-position gate of AC_ALGO_GATED (4 MiB of device
     * tables and a walk of the goto function to depth 10; built by default
     * where it applies). */
    AC_BUILD_NO_GATE = 4
};

typedef struct {
    uint64_t n_states;     /* states of the machine (trie nodes, root = 0) */
    uint32_t n_patterns;
    uint32_t sigma;        /* distinct bytes that occur in the patterns */
    uint32_t n_cols;       /* columns of the transition tables (>= sigma) */
    uint32_t m_max;        /* longest pattern, bytes */
    uint32_t placement;    /* resolved AC_PLACE_* used by AUTO scans */
    uint32_t hot_states;   /* rows in the LDS_HOT image (0 if none) */
    uint32_t class_shift;  /* byte -> column is (b >> shift) & (n_cols-1) when */
    uint32_t class_hashed; /*   class_hashed is 1; else a 256-entry map */
    uint64_t table_bytes;  /* device bytes of the DFA table (0 for goto-only) */
    uint64_t out_entries;  /* total entries of all output sets */
    double build_ms;       /* host time spent constructing the machine */
    uint32_t goto_only;    /* 1 if built with AC_BUILD_GOTO_ONLY */
    uint32_t pair_states;  /* states outside the LDS_HOT image with two-byte rows
                              (built with AC_BUILD_PAIR_ROWS); 0 if none */
    uint32_t has_gate;     /* start-position gate of AC_ALGO_GATED: 0 none, 1 the
                              class gate, 2 the hashed gate */
    double gate_pass;      /* expected share of start positions the gate passes (1.0
                              without a gate). Class gate: the fraction of the 4^10
                              window class strings it passes (uniformly random
                              text). Hashed gate: the chance that 6 bytes drawn with
                              the patterns' byte frequencies begin a pattern, plus
                              the filter's false-positive rate */
    double match_rate;     /* expected matches per text byte, for text whose bytes are
                              drawn independently with the patterns' own byte
                              frequencies (0 without a gate). Above 4e-3 the gated
                              scans stage matches in registers, reserving room in the
                              match list once per up to 512 matches per wavefront
                              (else once per up to 64) */
} ac_info_t;

/*
 * ac_build -- construct the machine for n_patterns patterns (Sec. II, step 1;
 * Sec. II.A for goto / failure / output functions; Sec. III for folding the
 * failure transitions into ordinary ones, giving a full DFA) and upload its
 * tables to the current device on `stream` (synchronised before return).
 *
 *   pat_bytes  host, concatenated pattern bytes
 *   pat_off    host, n_patterns + 1 non-decreasing offsets: pattern k is
 *              pat_bytes[pat_off[k] .. pat_off[k+1])
 *   opts       NULL for defaults
 *   out        receives the handle; free with ac_free
 *
 * Errors: AC_ERR_INVALID for n_patterns == 0, a null pointer, an empty
 * pattern or decreasing offsets; AC_ERR_TOO_LARGE if the table would need
 * 2^31 or more entries or the output sets 2^32 or more; AC_ERR_NOMEM,
 * AC_ERR_HIP.
 */
int ac_build(const uint8_t *pat_bytes, const uint64_t *pat_off, uint32_t n_patterns,
             const ac_build_opts *opts, void *stream, ac_automaton **out);

/*
 * ac_build_host -- the same construction as ac_build, kept on the host only
 * (no device is touched; ac_scan rejects the result). For inspecting the
 * tables with ac_get_table. Errors as ac_build, minus AC_ERR_HIP.
 */
int ac_build_host(const uint8_t *pat_bytes, const uint64_t *pat_off, uint32_t n_patterns,
                  const ac_build_opts *opts, ac_automaton **out);

/* Host tables of an automaton, in the library's state numbering (root = 0). */
enum {
    AC_TABLE_DFA = 0,     /* uint32 [n_states][n_cols]: successor | 1<<31 if it is final */
    AC_TABLE_GO = 1,      /* uint32 [n_states][n_cols]: goto child | 1<<31 if it ends a
                             pattern itself, 0 = no edge */
    AC_TABLE_OUT_OFF = 2, /* uint32 [n_states+1]: output set s = OUT_IDS[off[s] .. off[s+1]) */
    AC_TABLE_OUT_IDS = 3, /* uint32: pattern ids, ascending within each set */
    AC_TABLE_OWN_OFF = 4, /* uint32 [n_states+1]: patterns ending exactly at s */
    AC_TABLE_OWN_IDS = 5, /* uint32 */
    AC_TABLE_HOT_DFA = 6, /* uint16 [hot_states][n_cols] (plus one zero if the count is
                             odd): DFA rows of the LDS image, successor | 1<<15 if final */
    AC_TABLE_HOT_GO = 7,  /* uint16 [hot_states][n_cols]: goto rows of the LDS image */
    AC_TABLE_CMAP = 8,    /* uint8 [256]: byte -> column, 255 = byte in no pattern */
    AC_TABLE_PAIR = 9,    /* uint32 [pair_states][16]: row s - hot_states, column
                             c1 | c2 << 2 = state after classes c1, c2 from s,
                             | 1<<31 if the state after c1 is final (empty if none) */
    AC_TABLE_GATE_BITS = 10, /* uint32 [2^15]: bit x (word x >> 5, bit x & 31) is set
                                when a pattern can begin with a 10-byte window whose
                                classes, first byte in the lowest 2 bits, read x
                                (empty without a gate) */
    AC_TABLE_GATE_NODE = 11, /* uint32 [2^20]: per window code, the deepest goto state
                                its classes reach from the root: state | depth << 26,
                                | 1<<31 if a pattern ends on the path to it */
    AC_TABLE_PATH_OFF = 12,  /* uint32 [n_states+1]: patterns ending on the path from
                                the root to s (states of depth <= 10) ... */
    AC_TABLE_PATH_IDS = 13,  /* uint32: ... in PATH_IDS[off[s] .. off[s+1]), ascending */
    AC_TABLE_GATE2_BITS = 14, /* uint32 [2^11]: second gate level, bits
                                h = (y * 0x9E3779B1) >> 16 and (y * 0x85EBCA77) >> 16
                                (32-bit products) set for every class string y of 12
                                bytes (first byte in the lowest 2 bits) that a
                                pattern can begin with; a string passes when both of
                                its bits are set */
    AC_TABLE_QGATE_BITS = 15, /* uint32 [2^15]: hashed gate. For the first 6 bytes
                                b0..b5 of every pattern, X = b0 | b1 << 8 | b2 << 16,
                                Y = b3 | b4 << 8 | b5 << 16 and
                                h = X * 0x9E3779 + Y * 0x85EBCB (mod 2^32),
                                word h >> 17 has bits (h >> 12) & 31 and h & 31
                                set (empty without this gate) */
    AC_TABLE_QGATE_TAB = 16,  /* uint32 [slots][4], slots a power of two: one entry
                                per distinct 6-byte pattern start,
                                {X | (Y & 255) << 24, Y >> 8 | 1 << 31 | 1 << 30 if
                                patterns end at the goto state after the 6 bytes,
                                that state, its children (bit c set for an edge of
                                class c; all bits beyond 32 classes)}, in slot
                                (X * 0xC2B2AF ^ Y * 0x27D4EB) >> (32 - log2 slots)
                                or slot (X * 0x165667 ^ Y * 0xD3A2E5) >> (32 - log2
                                slots); unused slots are zero */
    AC_TABLE_OWN_ONE = 17,    /* uint32 [n_states] (with either gate, else empty): the
                                id of the one pattern ending exactly at s, or
                                0xffffffff when none or several do */
    AC_TABLE_PATH_ONE = 18    /* uint32 [n_states] (class gate, else empty): when
                                exactly one pattern ends on the path from the root
                                to s and its id is below 2^28, id | length << 28;
                                else 0xffffffff */
};

/*
 * ac_get_table -- copy host table `which` (AC_TABLE_*) into dst (host,
 * dst_bytes long) and store its size in *bytes. dst == NULL only queries
 * the size. Errors: AC_ERR_INVALID for an unknown table, a NULL automaton or
 * size pointer, or a destination that is too small.
 */
int ac_get_table(const ac_automaton *a, uint32_t which, void *dst, uint64_t dst_bytes,
                 uint64_t *bytes);

/* ac_free -- release the automaton and its device tables. NULL is a no-op.
 * The caller must ensure no scan using it is still running. */
void ac_free(ac_automaton *a);

/* ac_info -- sizes and choices of a built automaton. */
int ac_info(const ac_automaton *a, ac_info_t *info);

typedef struct {
    uint32_t algo;      /* AC_ALGO_* (default AUTO) */
    uint32_t chunk;     /* DFA: text bytes owned by one walker; multiple of 16;
                           0 = chosen from the text length */
    uint32_t block;     /* threads per workgroup; 0 = the placement's own (the only
                           value accepted otherwise) */
    uint32_t placement; /* 0 = the automaton's; else an AC_PLACE_* override */
    uint32_t walkers;   /* DFA: chunks walked in lockstep by each lane (1 to 4);
                           0 = auto */
    uint32_t block_bytes; /* DFA: text bytes a walker loads at once (64 or 128);
                             0 = auto */
    uint32_t pair_steps;  /* DFA, LDS_HOT: AC_PAIR_AUTO = a walker outside the image
                             looks up two bytes at once when the automaton was
                             built with AC_BUILD_PAIR_ROWS (ac_info_t.pair_states
                             > 0); AC_PAIR_OFF = one byte per lookup */
    uint32_t append;      /* 0 = *d_count is reset first; 1 = it is kept and the new
                             matches go after the ones it counts (several scans
                             then fill one list, and no reset runs on the stream) */
} ac_scan_opts;

enum { AC_PAIR_AUTO = 0, AC_PAIR_OFF = 1 };

/*
 * ac_scan -- process the text with the machine in one pass (Sec. II, step 2)
 * and append every match to d_matches. Asynchronous on `stream`.
 *
 * With AC_ALGO_DFA the text is split into chunks of `chunk` bytes; the walker
 * of chunk [kC, kC + C) starts max(0, kC - m_max + 1) bytes in (rounded down
 * to 16) from the root and reports only matches ending inside its chunk, so
 * every occurrence is reported exactly once. With AC_ALGO_PFAC every start
 * position gets its own failure-less walk (Sec. II.B, Sec. IV.A); with
 * AC_ALGO_GATED only the start positions the gate passes do, so each
 * occurrence is again reported once, by the walk from its first byte.
 *
 *   d_text     device, n bytes, 16-byte aligned (n == 0 allowed)
 *   d_matches  device, room for `capacity` uint64 keys
 *   d_count    device uint64; set to the total number of matches, even when
 *              it exceeds capacity (only the first `capacity` keys written)
 *   opts       NULL for defaults
 *
 * Errors (checked before anything is queued): AC_ERR_INVALID for null
 * pointers, a misaligned text or bad options; AC_ERR_TOO_LARGE for
 * n >= 2^32; AC_ERR_HIP if a launch fails. Overflow is not an error here:
 * compare *d_count with capacity, or use ac_scan_sync.
 */
int ac_scan(const ac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_matches,
            uint64_t capacity, uint64_t *d_count, const ac_scan_opts *opts, void *stream);

/*
 * ac_scan_stream -- continue a text that arrives in pieces (the per-buffer
 * search of the paper's Alg. 1, with the machine's state carried from one
 * buffer to the next, so occurrences that span pieces are found).
 * Asynchronous on `stream`; DFA scan only.
 *
 *   d_text, n     device, this piece (16-byte aligned)
 *   base          position of the piece's first byte in the whole text;
 *                 matches are reported as (base + local end) << 32 | id,
 *                 and base + n must stay below 2^32
 *   d_state_in    device uint32: the state the previous piece ended in, as
 *                 written to its d_state_out; NULL for the first piece (root)
 *   d_state_out   device uint32 (NULL = not wanted): receives the state after
 *                 the piece's last byte. The value is an opaque token of this
 *                 automaton. Must not alias d_state_in.
 *   append        nonzero: add to *d_count and the keys already in d_matches
 *                 instead of starting from zero (one list for all pieces)
 *
 * Errors: as ac_scan, plus AC_ERR_INVALID for an algo other than
 * AC_ALGO_DFA or aliased state words.
 */
int ac_scan_stream(const ac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t base,
                   const uint32_t *d_state_in, uint32_t *d_state_out, uint64_t *d_matches,
                   uint64_t capacity, uint64_t *d_count, int append, const ac_scan_opts *opts,
                   void *stream);

/*
 * ac_scan_sync -- ac_scan, then wait for `stream` and copy the total count to
 * *h_count. Returns AC_ERR_OVERFLOW if the total exceeds capacity (the first
 * `capacity` keys are still valid).
 */
int ac_scan_sync(const ac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_matches,
                 uint64_t capacity, uint64_t *d_count, const ac_scan_opts *opts, void *stream,
                 uint64_t *h_count);

/*
 * ac_sort_matches -- sort `count` keys in place, ascending, on `stream`,
 * giving the canonical (e, k) order. d_tmp is device scratch of at least
 * ac_sort_scratch_bytes(count) bytes, owned by the caller.
 * Errors: AC_ERR_INVALID for null pointers or too small scratch.
 */
uint64_t ac_sort_scratch_bytes(uint64_t count);
int ac_sort_matches(uint64_t *d_keys, uint64_t count, void *d_tmp, uint64_t tmp_bytes,
                    void *stream);

/* ------------------------------------------------------------------ batches
 * Many texts against several resident automata in one persistent launch. The
 * texts live in one device buffer (the "batch buffer"); text t occupies bytes
 * [text_off[t], text_off[t] + text_len[t]) of it and is matched against
 * automaton text_auto[t]. Matches are reported as
 * (end position in the batch buffer << 32) | pattern id of that text's
 * automaton, so the batch buffer must be shorter than 2^32 bytes. Each
 * text's list equals what ac_scan reports for it alone, shifted by its offset.
 */
typedef struct ac_batch ac_batch;

typedef struct {
    uint32_t placement; /* DFA: AC_PLACE_AUTO (LDS_HOT when every automaton has an
                           LDS image, else GLOBAL), AC_PLACE_LDS_HOT or AC_PLACE_GLOBAL */
    uint32_t walkers;   /* DFA: chunks walked per lane (1 to 4); 0 = by placement */
    uint32_t chunk;     /* DFA: end positions per work item; gated: start positions
                           per task (rounded to whole 1,008-byte tiles); 0 = from
                           the batch size */
    uint32_t algo;      /* ac_batch_create: AC_ALGO_AUTO (GATED when every automaton
                           has the class gate and AC_ALGO_AUTO would pick GATED for
                           it, else DFA), AC_ALGO_DFA or AC_ALGO_GATED (the gated
                           failure-less scan, tasks of whole tiles of one text taken
                           from a device counter, LDS bitmaps loaded per automaton).
                           ac_scan_batch: AUTO or DFA */
} ac_batch_tune;

typedef struct {
    uint32_t placement, walkers, block_bytes, chunk;  /* DFA plans; gated: 0, 0, 0, task bytes */
    uint32_t threads;  /* per workgroup */
    uint32_t grid;     /* workgroups of the persistent launch */
    uint32_t n_items;  /* work items (chunks of texts; gated: tasks) */
    uint32_t n_tasks;  /* runs of items of one automaton, split over the grid */
    uint64_t text_bytes;
    uint32_t algo;     /* AC_ALGO_DFA or AC_ALGO_GATED */
    uint32_t pad;
} ac_batch_info_t;

/*
 * ac_batch_create -- plan a batch: cut every text into work items, order them
 * by automaton, upload the plan (on `stream`, synchronised before return).
 *
 *   autos, n_autos    automata built with ac_build on the current device, all
 *                     with the same byte-class scheme (ac_info: class_hashed and
 *                     n_cols); for AC_PLACE_LDS_HOT build them with
 *                     placement AC_PLACE_LDS_HOT so each has an image
 *   text_off          host, n_texts offsets into the batch buffer, multiples of 16
 *   text_len          host, n_texts lengths (0 allowed)
 *   text_auto         host, n_texts automaton indices
 *   tune              NULL for defaults (see ac_batch_tune)
 *   out               receives the plan; free with ac_batch_free
 *
 * The automata must outlive the plan. Errors: AC_ERR_INVALID (NULL arrays,
 * misaligned offsets, an index past n_autos, mixed class schemes, a placement
 * the automata cannot use), AC_ERR_TOO_LARGE (buffer of 2^32 bytes or more),
 * AC_ERR_NOMEM, AC_ERR_HIP.
 */
int ac_batch_create(const ac_automaton *const *autos, uint32_t n_autos, const uint64_t *text_off,
                    const uint64_t *text_len, const uint32_t *text_auto, uint32_t n_texts,
                    const ac_batch_tune *tune, void *stream, ac_batch **out);

/* ac_batch_info -- the plan's resolved choices and sizes. */
int ac_batch_info(const ac_batch *b, ac_batch_info_t *info);

/*
 * ac_batch_scan -- reset *d_count and scan the whole batch in one launch on
 * `stream` (asynchronous). d_texts: device batch buffer, 16-byte aligned,
 * covering every text of the plan. With use_graph nonzero the reset and the
 * launch are captured into a hipGraph on the first call (and again whenever
 * the buffer arguments change) and replayed on `stream` afterwards.
 * Overflow is reported as by ac_scan: *d_count holds the true total.
 * The plan holds the launch's task counter, so scans of one plan must not
 * overlap (issue them on one stream, or synchronise between streams).
 */
int ac_batch_scan(ac_batch *b, const uint8_t *d_texts, uint64_t *d_matches, uint64_t capacity,
                  uint64_t *d_count, int use_graph, void *stream);

/* ac_batch_free -- release the plan and its graph; call it after the plan's
 * last scan has completed. NULL is a no-op. */
void ac_batch_free(ac_batch *b);

/*
 * ac_scan_batch -- one-shot form, with the text descriptors in device memory:
 * plan, scan and free in one call (Sec. III's input split, applied to many
 * texts, each against its own machine, Sec. IV.A). Text t is bytes
 * [d_text_off[t], d_text_off[t+1]) of the batch buffer d_texts and is matched
 * against autos[d_text_auto[t]]. The work items are planned on the device
 * (chunks of every text, ordered by automaton), so the descriptors never
 * visit the host.
 *
 *   d_texts       device batch buffer, 16-byte aligned
 *   d_text_off    device, n_texts + 1 non-decreasing uint64 offsets; each
 *                 non-empty text starts at a multiple of 16; the last offset
 *                 is below 2^32
 *   d_text_auto   device, n_texts uint32 indices into autos
 *   d_match_text  device, room for `capacity` uint32 (NULL = not wanted):
 *                 receives, beside each key written to d_matches, the index
 *                 of the text the match lies in
 *   d_matches, capacity, d_count  keys as ac_batch_scan (end positions in
 *                 the batch buffer); *d_count holds the true total
 *   tune          NULL for defaults (placement, walkers, chunk)
 *
 * Device scratch for the plan (about 17 MB plus 4 bytes per text) is
 * allocated and freed by the call. Synchronises `stream` before returning.
 * Errors: AC_ERR_INVALID for NULL pointers, an unaligned buffer, automata
 * that cannot share a launch, and (found by the device plan) decreasing
 * offsets, unaligned text starts or an automaton index past n_autos;
 * AC_ERR_TOO_LARGE for more than 2^19 texts or a buffer of 2^32 bytes or
 * more; AC_ERR_NOMEM; AC_ERR_HIP.
 */
int ac_scan_batch(const ac_automaton *const *autos, uint32_t n_autos, const uint8_t *d_texts,
                  const uint64_t *d_text_off, const uint32_t *d_text_auto, uint32_t n_texts,
                  uint32_t *d_match_text, uint64_t *d_matches, uint64_t capacity, uint64_t *d_count,
                  const ac_batch_tune *tune, void *stream);

/*
 * ac_scan_batch_noalloc -- ac_scan_batch for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid allocation): the same arguments and results, with the plan in
 * a scratch array of fixed size inside the library (one per GPU, held until
 * the process ends) instead of a buffer allocated per call. It calls no
 * hipMalloc or hipFree.
 *
 * Limits: at most 65,536 texts (AC_ERR_TOO_LARGE beyond); the scratch holds
 * up to 2^20 work items, and the chunk length grows to stay within that.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (on different streams, or from threads that do not wait for each
 * other) race on it and must not be made; calls from several host threads
 * take turns on the host side. Synchronises `stream` before returning.
 * Errors as ac_scan_batch, minus AC_ERR_NOMEM.
 */
int ac_scan_batch_noalloc(const ac_automaton *const *autos, uint32_t n_autos, const uint8_t *d_texts,
                          const uint64_t *d_text_off, const uint32_t *d_text_auto, uint32_t n_texts,
                          uint32_t *d_match_text, uint64_t *d_matches, uint64_t capacity, uint64_t *d_count,
                          const ac_batch_tune *tune, void *stream);

/* ------------------------------------------------------------------ serving
 * A request loop over resident automata with continuous batching: requests
 * are admitted while others are on the device, as slots (one HIP stream
 * each) and a device-memory budget allow, and their scans overlap on the
 * GPU. A request's work runs on its slot's stream alone; streams that share
 * a hardware queue run their kernels in turn, so the process should have at
 * least as many hardware queues as slots (HIP reads GPU_MAX_HW_QUEUES at
 * start-up; its default is 4). Automata the gated
 * scan suits (AC_ALGO_AUTO's rule) scan a request in one gated launch; the
 * others in pieces with the DFA state carried on the device from one piece to
 * the next (the per-buffer search of the paper's Alg. 1). Either way a
 * request's match list equals what ac_scan reports for the same text alone.
 */
typedef struct ac_server ac_server;

typedef struct {
    uint64_t hbm_budget;   /* device bytes for request text copies and match lists
                              (one allocation at create); 0 = 4 GiB */
    uint32_t max_inflight; /* requests on the device at once (slots, <= 64); 0 = 8 */
    uint32_t piece_bytes;  /* scan piece length, a multiple of 16; 0 = 16 MiB */
    uint32_t match_ppm;    /* first guess of matches per million text bytes, used to
                              size match lists until finished requests refine it;
                              0 = 20000. A low guess costs a rescan, never a result. */
    uint32_t flags;        /* reserved, must be 0 */
    uint32_t max_large;    /* at most this many requests of 4 MiB or more on the device at
                              once (each fills the GPU by itself); shorter requests are
                              admitted past one that waits for this. 0 = no limit:
                              on the served benchmark's mix overlapping them is faster
                              (2: 690 GB/s, 1: 463, none: 711) */
    uint32_t reserved;     /* must be 0 */
} ac_serve_opts;

typedef struct {
    int32_t status;           /* AC_OK or the error that ended the request */
    uint32_t automaton;
    uint64_t n;               /* text bytes */
    const uint64_t *d_matches; /* device keys (end << 32 | id, end relative to the
                                  request's text), unordered; valid until
                                  ac_serve_release */
    uint64_t n_matches;
    uint64_t t_submit_ns, t_admit_ns, t_done_ns; /* arrival, admission and completion,
                                                    on the server's clock */
    uint32_t pieces;          /* scan launches of the last run (1 for a gated scan) */
    uint32_t rescans;         /* scans repeated because the list was too small */
} ac_serve_result;

typedef struct {
    uint64_t submitted, completed, failed, queued, running, rescans;
    uint64_t pool_bytes, pool_used, pool_peak;
    uint64_t running_peak;  /* most requests on the device at once */
    uint64_t bytes_done;    /* text bytes of successfully finished requests */
    double p50_ms, p99_ms;  /* latency (arrival to completion) of the last finished
                               requests, up to 65,536 of them; 0 if none */
    double gbps;            /* bytes_done / (last completion - first arrival) */
} ac_serve_stats_t;

/*
 * ac_serve_create -- start a server on the current device over n_autos
 * automata built with ac_build (they must outlive the server). Allocates the
 * device pool and the slots and starts the scheduler thread.
 * Errors: AC_ERR_INVALID, AC_ERR_NOMEM (pool), AC_ERR_HIP.
 */
int ac_serve_create(const ac_automaton *const *autos, uint32_t n_autos, const ac_serve_opts *opts,
                    ac_server **out);

/* ac_serve_add -- make one more automaton (built with ac_build on the
 * server's device) resident; *id receives its index for ac_serve_submit. */
int ac_serve_add(ac_server *s, const ac_automaton *a, uint32_t *id);

/*
 * ac_serve_submit -- queue a scan of `text` (n bytes) with automaton
 * `automaton`; returns at once with a ticket. arrival_ns = 0 means the request
 * arrives now; a later time on the server's clock (ac_serve_now_ns) schedules
 * its arrival, so that a recorded or generated arrival process can be
 * replayed exactly: nothing is admitted before its arrival, and latency
 * counts from it (t_submit_ns). With text_on_device nonzero the
 * text is device memory (16-byte aligned), already written when the call is
 * made (work queued on other streams to produce it must have completed: the
 * server's streams do not wait on the caller's), and unchanged until the
 * request is done; otherwise it is host memory that the server copies into
 * its pool (pinned memory copies without blocking the scheduler), and that
 * must stay valid until the request is done.
 * Errors: AC_ERR_INVALID; AC_ERR_TOO_LARGE if n >= 2^32 or the request alone
 * exceeds the budget.
 */
int ac_serve_submit(ac_server *s, uint32_t automaton, const uint8_t *text, uint64_t n, int text_on_device,
                    uint64_t arrival_ns, uint64_t *ticket);

/* ac_serve_now_ns -- the server's clock: nanoseconds since ac_serve_create. */
uint64_t ac_serve_now_ns(const ac_server *s);

/*
 * ac_serve_wait -- block until the request is done (timeout_ms < 0: no limit)
 * and describe it in *res. Returns AC_ERR_BUSY on timeout, the request's own
 * error if it failed, else AC_OK. May be called again for the same ticket.
 */
int ac_serve_wait(ac_server *s, uint64_t ticket, int64_t timeout_ms, ac_serve_result *res);

/* ac_serve_release -- give back a finished request's match list to the pool
 * (a result not released keeps its bytes of the budget). */
int ac_serve_release(ac_server *s, uint64_t ticket);

/* ac_serve_stats -- counters and pool occupancy. */
int ac_serve_stats(ac_server *s, ac_serve_stats_t *st);

/* ac_serve_destroy -- finish what is on the device, fail what is still
 * queued with AC_ERR_BUSY, stop the thread and free everything (unreleased
 * match lists included). NULL is a no-op. */
void ac_serve_destroy(ac_server *s);

/* ------------------------------------------------------------- measurement
 * Streaming kernels of known traffic that the scans are priced against. They
 * match nothing.
 *
 * ac_hbm_read -- read the n bytes at device pointer d (16-byte aligned) once,
 * with the scans' 16-byte non-temporal loads over the whole GPU, and
 * XOR-accumulate them into *d_fold as 32-bit little-endian words (a short
 * last word zero-padded): *d_fold ^= fold. The time of one call on a buffer
 * far larger than the caches is the HBM read ceiling.
 * ac_hbm_copy -- copy n bytes from src to dst (device, 16-byte aligned, not
 * overlapping) with the same loads and non-temporal stores: a kernel that
 * reads n and writes n bytes, for scaling HBM byte counters.
 * `blocks` is the workgroup count (256 threads each); 0 picks one per
 * compute unit. Both are asynchronous on `stream`.
 * Errors: AC_ERR_INVALID for NULL or unaligned pointers, overlapping copies;
 * AC_ERR_HIP for a failed launch.
 */
int ac_hbm_read(const void *d, uint64_t n, uint64_t *d_fold, uint32_t blocks, void *stream);
int ac_hbm_copy(void *dst, const void *src, uint64_t n, uint32_t blocks, void *stream);

/* ac_last_error -- message of the last failing call on this thread ("" if none). */
const char *ac_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AC_H */
