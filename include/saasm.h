/*
 * saasm.h -- C ABI of the MI355X (gfx950) suffix-array / read-overlap library.
 *
 * The library builds the suffix array of shotgun fragments laid end to end (each fragment
 * closed by its own '$' separator), the LCP array beside it, and the longest suffix-prefix
 * overlap of every ordered pair of fragments, with hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless the name ends in _h (host memory).
 *  - Memory: the caller allocates every buffer, including the scratch workspace `ws`.  The
 *    library never allocates device memory inside these calls and never frees caller memory.
 *    Workspace contents are scratch: nothing is carried from one call to the next.
 *  - Streams: every call is ordered on `stream`.  Calls that report a count or status to the
 *    host (sa_build, sa_build_dc3, sa_overlaps, sa_lookup, sa_pack, sa_sort_pairs,
 *    sa_revcomp_text, sa_strand_rows) synchronise `stream` before they return; sa_lcp does not.
 *  - Errors: every call returns an int status (SA_OK or a negative SA_ERR_*) and never throws
 *    across the ABI.  sa_last_error() returns a message for the calling thread's last failure.
 *    On error the outputs are unspecified; inputs are never modified.
 *  - Thread safety: calls are re-entrant as long as concurrent calls use different workspaces.
 *  - Text: bytes 'A','C','G','T' and '$'; text[n-1] must be '$'.  Read i is the bytes between
 *    the (i-1)-th and i-th separator (empty reads, "$$", are allowed).  Positions are offsets
 *    in the text, separators included; read ids count separators from 0.
 *  - Size: 1 <= n <= 2^31 - 3 (positions, ranks and counts are 32-bit).
 *
 * Ordering (Sec. IV of the paper: the suffix array is the sorted array of all suffixes of the
 * text; Sec. III: the text is the set of shotgun fragments): the separator closing read i
 * sorts below the one closing read j when i < j, every separator sorts below every base, and
 * A < C < G < T.  With distinct separators all suffixes differ, so the suffix array is unique.
 */
#ifndef SAASM_H
#define SAASM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SA_OK = 0,
    SA_PENDING = 1,          /* asynchronous work not finished yet */
    SA_ERR_INVALID = -1,     /* bad argument: NULL pointer, text not ending in '$', bad tuning */
    SA_ERR_ALPHABET = -2,    /* a byte other than A, C, G, T, '$' */
    SA_ERR_TOO_LARGE = -3,   /* n > 2^31 - 3 */
    SA_ERR_NOMEM = -4,       /* workspace too small (the required size is reported) */
    SA_ERR_CAPACITY = -5,    /* output buffer too small (the required count is reported) */
    SA_ERR_HIP = -6,         /* a HIP runtime call or a kernel's own consistency check failed */
    SA_ERR_NOTFOUND = -7     /* unknown job id or timing key */
};

/* Launch tuning of the radix sort; a zero field means "use the default".
 *   digit_bits       4, 8, 9 or 11 bits per LSD pass (default 9)
 *   block_threads    256, 512 or 1024 threads per workgroup (4, 8 or 16 wave64 wavefronts;
 *                    1024 only with 16 items and digit_bits <= 9; default 1024, or 512 for
 *                    11-bit digits)
 *   items_per_thread 8 or 16 keys per thread (tile = block_threads * items_per_thread)
 *   seg_pack         sa_build_batched only: at most this many characters per build
 *                    (consecutive texts are packed greedily; 0 = all texts in one build);
 *                    must be 0 for the other entry points                                 */
typedef struct {
    int32_t digit_bits;
    int32_t block_threads;
    int32_t items_per_thread;
    int32_t seg_pack;
} sa_tuning;

/* Library version string (static storage). */
const char *sa_version(void);

/* Message describing the calling thread's most recent error (static per-thread storage). */
const char *sa_last_error(void);

/* ---------------------------------------------------------------------------------------- */
/* Validation and 2-bit packing.  Sec. III: DNA is a string over the four bases A, C, G, T;    */
/* the fragments are laid end to end, each followed by its separator.                         */
/* ---------------------------------------------------------------------------------------- */

/* Words of packed output for a text of n bytes (each array is padded for over-reads). */
int64_t sa_packed_words(int64_t n);   /* uint32 words of 2-bit codes, 16 bases per word       */
int64_t sa_sepmask_words(int64_t n);  /* uint32 words of separator bits, 32 positions per word */

/* Workspace bytes for sa_pack. */
int64_t sa_pack_ws_bytes(int64_t n);

/* sa_pack: validate the text and pack it.
 *   text      [n] bytes
 *   packed    [sa_packed_words(n)] out: base j of word w is position 16w+j, stored in bits
 *             (31-2j, 30-2j), A=0 C=1 G=2 T=3; a separator packs as 0; padding is 0
 *   sepmask   [sa_sepmask_words(n)] out: bit (31-j) of word w is set when position 32w+j is '$'
 *   read_end  [cap_reads] out, may be NULL: position of the separator closing each read
 *   m_h       host out: number of reads (separators)
 * Returns SA_ERR_ALPHABET / SA_ERR_INVALID for a bad text, SA_ERR_CAPACITY (with *m_h set) when
 * read_end is given and cap_reads < m.  Synchronises the stream. */
int sa_pack(const uint8_t *text, int64_t n, uint32_t *packed, uint32_t *sepmask,
            int32_t *read_end, int64_t cap_reads, int64_t *m_h, void *ws, int64_t ws_bytes,
            hipStream_t stream);

/* ---------------------------------------------------------------------------------------- */
/* Radix sort (Sec. IV: LSD radix sort, each pass a counting sort in which an element's output */
/* index is the number of elements in lower buckets plus those already in its own bucket;      */
/* per pass: per-tile digit counts, a prefix sum over the (digit x tile) table, and a scatter).*/
/* ---------------------------------------------------------------------------------------- */

/* Workspace bytes for sa_sort_pairs on n pairs. */
int64_t sa_sort_ws_bytes(int64_t n, const sa_tuning *tune_or_null);

/* sa_sort_pairs: stable sort of (key, value) pairs by bits [bit_lo, bit_hi) of the key.
 *   keys, vals  [n] in/out: sorted in place (the library copies back when the result ends up
 *               in its workspace)
 *   0 <= bit_lo < bit_hi <= 64.  Equal digits keep their input order (stability), so bits
 *   outside the range keep the order they had.  Synchronises the stream. */
int sa_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi,
                  void *ws, int64_t ws_bytes, const sa_tuning *tune_or_null, hipStream_t stream);

/* ---------------------------------------------------------------------------------------- */
/* Suffix array (Sec. IV), by prefix doubling over LSD radix sorts of rank-pair keys.          */
/* A doubling round whose groups all have at most 32 members orders each group in on-chip    */
/* memory instead of running radix passes over all its keys; the result is the same.         */
/* ---------------------------------------------------------------------------------------- */

/* Workspace bytes for sa_build on a text of n bytes. */
int64_t sa_build_ws_bytes(int64_t n, const sa_tuning *tune_or_null);

/* One workspace for the whole path on a text of n bytes with at most n_reads_upper reads
 * (<= 0: assume n): the largest of what sa_build (default tuning), sa_lcp and sa_overlaps need,
 * the last with room for up to n candidate matches of its walks (a text with more makes
 * sa_overlaps return SA_ERR_NOMEM with the size it needs).  The calls may share it because each
 * finishes with it before the next starts on the same stream.  -1 for n < 1. */
int64_t sa_workspace_bytes(int64_t n, int64_t n_reads_upper);

/* sa_build: suffix array of the text.
 *   text         [n] bytes (see conventions)
 *   sa           [n] out: the permutation of 0..n-1 listing suffixes in sorted order
 *   isa_or_null  [n] optional out: inverse permutation, isa[sa[i]] == i
 *   rounds_h     optional host out: number of sort rounds run (first sort + doubling rounds)
 * Synchronises the stream once per round. */
int sa_build(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
             void *ws, int64_t ws_bytes, const sa_tuning *tune_or_null, int32_t *rounds_h,
             hipStream_t stream);

/* The same suffix array by the skew recursion over the difference cover {1, 2} mod 3 (the
 * linear-work construction of Kärkkäinen, Sanders and Burkhardt that Sec. IV cites and names
 * its radix-sort kernel after): the samples (positions not 0 mod 3) are sorted by their first
 * three symbols with the radix passes of sa_sort_pairs and named, the string of names is
 * sorted recursively while two samples share a name, the other suffixes are sorted by
 * (symbol, rank of the next suffix), and the two lists are merged.  Arguments, layout and
 * errors are those of sa_build; the output is identical to sa_build's.
 *   levels_h     optional host out: number of recursion levels run (1 = no recursion)
 * The workspace is about 72 bytes per character (sa_build: about 45).  Synchronises the stream
 * once per level. */
int64_t sa_build_dc3_ws_bytes(int64_t n, const sa_tuning *tune_or_null);
int sa_build_dc3(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
                 void *ws, int64_t ws_bytes, const sa_tuning *tune_or_null, int32_t *levels_h,
                 hipStream_t stream);

/* Batched build of many independent texts in one set of launches (the fragment sets of
 * Sec. III, one per assembly job).  The texts are laid end to end in `text`; text s occupies
 * text[set_off_h[s] .. set_off_h[s+1]) and must end with '$'.
 *   set_off_h   host [n_sets+1]: 0 = set_off_h[0] < ... < set_off_h[n_sets] = n
 *   sa          [n] out: for every s, sa[set_off_h[s] .. set_off_h[s+1]) is the suffix array
 *               of text s, in concatenated coordinates (subtract set_off_h[s] for local ones)
 *   isa_or_null [n] optional out: inverse of sa
 *   lcp_or_null [n] optional out: the LCP array of each text in its block (lcp[set_off_h[s]]
 *               is 0); the same array sa_lcp gives for the concatenated text.  A failure found
 *               while computing it is reported the way sa_lcp reports it (in lcp[0]).
 *   use_graph   nonzero: the doubling rounds are recorded once as a hipGraph and replayed
 * The workspace size depends on the packing when tune->seg_pack > 0: pass the same offsets to
 * sa_build_batched_ws_bytes (NULL offsets give the size for one build of all texts); it
 * includes the room the LCP needs.  sa_lcp and sa_overlaps accept the concatenated text with
 * this sa/isa unchanged: LCP is 0 at every block start and no overlap pairs reads of different
 * texts.  Synchronises the stream once per round (once per graph replay). */
int64_t sa_build_batched_ws_bytes(int64_t n, int32_t n_sets, const int64_t *set_off_h_or_null,
                                  const sa_tuning *tune_or_null);
int sa_build_batched(const uint8_t *text, int64_t n, const int64_t *set_off_h, int32_t n_sets,
                     int32_t *sa, int32_t *isa_or_null, int32_t *lcp_or_null, void *ws,
                     int64_t ws_bytes, const sa_tuning *tune_or_null, int32_t use_graph,
                     int32_t *rounds_h, hipStream_t stream);

/* ---------------------------------------------------------------------------------------- */
/* LCP array beside the suffix array (Kasai's permuted-LCP scan; the paper uses the array for  */
/* prefix matching between fragments, Sec. IV).                                              */
/* ---------------------------------------------------------------------------------------- */

int64_t sa_lcp_ws_bytes(int64_t n);

/* sa_lcp: lcp[0] = 0 and lcp[i] = length of the common prefix of the suffixes at sa[i-1] and
 * sa[i]; separators never match.  sa and isa must come from sa_build on the same text
 * (isa[sa[i]] == i).  Does not synchronise, so failures that only the device can see (a byte
 * other than A, C, G, T, '$'; a text without its final '$'; sa/isa entries out of range) are
 * reported in the output: lcp[0] then holds the negative status (SA_ERR_ALPHABET,
 * SA_ERR_INVALID or SA_ERR_HIP) instead of 0.  sa_lcp_status reads it; sa_overlaps returns it. */
int sa_lcp(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa,
           int32_t *lcp, void *ws, int64_t ws_bytes, hipStream_t stream);

/* sa_lcp_noalloc: sa_lcp for callers that cannot allocate (code under stream capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, result and error
 * reporting as sa_lcp, but no workspace argument: the scratch is one array of 18 MiB that the
 * library holds in every GPU's memory until the process ends, so 1 <= n <= 2^24
 * (sa_lcp_noalloc_max_n(); larger n: SA_ERR_TOO_LARGE).  Allocates nothing (no device, pinned
 * or host memory on success, no timing events).  Every call on one GPU uses that GPU's array:
 * calls that overlap in time on one GPU (other streams, other host threads) race, so the
 * caller orders them; one stream orders them by itself. */
int64_t sa_lcp_noalloc_max_n(void);
int sa_lcp_noalloc(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa,
                   int32_t *lcp, hipStream_t stream);

/* sa_lcp_status: synchronises `stream` and returns the status an earlier sa_lcp (or
 * sa_build_batched with an LCP output) on that stream left in lcp[0]: SA_OK when it is 0. */
int sa_lcp_status(const int32_t *lcp, hipStream_t stream);

/* Positions scanned per thread by sa_lcp: 1, 2, 4, 8 or 16 (each thread restarts Kasai's
 * carried bound at its first position; any value gives the same result).  Process-wide;
 * default 4. */
int sa_lcp_set_chunk(int32_t chunk);

/* Size from which sa_lcp stores the scan's lengths by text position first and then gathers
 * lcp[i] = plcp[sa[i]], instead of writing lcp[isa[p]] at random: above the last-level cache
 * (about 64 M positions of 4-byte lengths) a random gather costs about half a random scatter.
 * The workspace then holds n more int32 (sa_lcp_ws_bytes accounts for it).  Both forms give
 * the same array.  min_n >= 0 sets it (process-wide; size workspaces after setting it) and
 * returns the previous value; min_n < 0 only returns the current one (default 2^26). */
int64_t sa_lcp_plcp_min(int64_t min_n);

/* ---------------------------------------------------------------------------------------- */
/* Pattern lookup (Sec. IV: the suffix array is searched to decide whether a string -- e.g. a  */
/* fragment -- is a prefix of a suffix of the text).                                          */
/* ---------------------------------------------------------------------------------------- */

/* Workspace bytes for sa_lookup on a text of n bytes with patterns of pat_total bytes in all. */
int64_t sa_lookup_ws_bytes(int64_t n, int64_t pat_total);

/* sa_lookup: for each pattern P_i = pat[pat_off[i] .. pat_off[i+1]) over A, C, G, T, the
 * interval [lo, hi) of suffix-array indices whose suffixes start with P_i:
 *   lohi[2i] = lo  = number of suffixes that sort below P_i without starting with it,
 *   lohi[2i+1] = hi, so hi - lo = number of positions where P_i occurs in the text.
 * An empty pattern gives [0, n).  Patterns never match across a separator.
 *   text     [n] the text sa was built from
 *   sa       [n] from sa_build on that text
 *   pat      [pat_total] pattern bytes, concatenated (may be NULL when pat_total == 0)
 *   pat_off  [n_pat + 1] int64, non-decreasing, pat_off[0] >= 0, pat_off[n_pat] <= pat_total
 *   lohi     [2 * n_pat] int32 out
 * Errors: SA_ERR_ALPHABET when a pattern (or the text) holds another byte; SA_ERR_INVALID for
 * offsets out of range or a text without its final '$'.  Synchronises the stream. */
int sa_lookup(const uint8_t *text, int64_t n, const int32_t *sa, const uint8_t *pat,
              const int64_t *pat_off, int64_t pat_total, int32_t n_pat, int32_t *lohi,
              void *ws, int64_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------- */
/* Reconstruction from the fragments of two cuttings ("cut and continue", Sec. III), its       */
/* prefix tests answered by searching the suffix array (Sec. IV).                            */
/* ---------------------------------------------------------------------------------------- */

/* sa_reconstruct: HOST function.  The text's reads are the fragments of a sequence S cut twice
 * at disjoint sets of interior positions, mixed (read i = fragment i).  Starting from a 'fir'
 * pair (a fragment that is a proper prefix of another: the first pieces of the two cuttings),
 * the cutting that is behind repeatedly takes a fragment that starts with the remainder (the
 * part of S known beyond it) or is a proper prefix of the remainder; a dead end goes back to
 * the last choice.  Pairs are tried by the longer fragment's id, then the shorter's; later
 * choices in increasing fragment id; the first complete reconstruction is returned.  Candidate
 * fragments are found by walking the suffix array from the remainder's rank under the running
 * LCP minimum.
 *   text_h, n          the fragments, each closed by '$' (no empty fragment), host memory
 *   sa_h, isa_h, lcp_h  sa_build / sa_lcp results for that text, copied to host memory
 *   order_h            [m] out: fragment ids in placement order
 *   rs_h               [rs_cap] out, may be NULL: the reconstructed sequence
 *   rs_len_h           out: its length
 *   max_steps          bound on search steps
 * Returns SA_OK; SA_ERR_NOTFOUND when no reconstruction exists (or max_steps is reached);
 * SA_ERR_CAPACITY when rs_cap is too small; SA_ERR_INVALID for inconsistent input. */
int sa_reconstruct(const uint8_t *text_h, int64_t n, const int32_t *sa_h, const int32_t *isa_h,
                   const int32_t *lcp_h, int32_t *order_h, uint8_t *rs_h, int64_t rs_cap,
                   int64_t *rs_len_h, int64_t max_steps);

/* sa_overlap_path: HOST function.  Sec. III reads a reconstruction off a weighted directed
 * graph: one vertex per fragment, an edge a -> b weighted by the overlap length l(a, b), and the
 * superstring obtained by merging the fragments along a Hamiltonian path of maximal total
 * weight (each next fragment contributes what lies past its overlap with the one before).
 *   text_h, n     the fragments, each closed by '$' (host memory; any bytes besides '$')
 *   rows_h, r     [r][3] host rows (a, b, l): the edges, e.g. sa_overlaps' output copied to the
 *                 host; any order; pairs without a row weigh 0
 *   exact_max_m   m <= exact_max_m (at most 20): exact search, dynamic programming over subsets
 *                 of fragments (2^m * m^2 steps, 9 * 2^m * m bytes of host memory); among paths
 *                 of equal weight the one found first (subsets in increasing order, fragments in
 *                 increasing id) ending at the smallest id.  Larger m: the greedy rule -- edges
 *                 by weight (heaviest first, then by a, then by b), an edge kept when a has no
 *                 successor yet, b no predecessor and the two are not in one chain already; the
 *                 chains laid end to end in order of their first fragment.
 *   order_h       [m] out: fragment ids along the path
 *   weight_h      out: the path's total weight
 *   rs_h          [rs_cap] out, may be NULL when rs_cap is 0: the merged superstring
 *   rs_len_h      out: its length
 * Returns SA_ERR_INVALID for rows that name fragments out of range, a == b, or a length above
 * either fragment's; SA_ERR_CAPACITY (order, weight and *rs_len_h set) when rs_cap is too small. */
int sa_overlap_path(const uint8_t *text_h, int64_t n, const int32_t *rows_h, int64_t r,
                    int32_t exact_max_m, int32_t *order_h, int64_t *weight_h, uint8_t *rs_h,
                    int64_t rs_cap, int64_t *rs_len_h);

/* ---------------------------------------------------------------------------------------- */
/* Suffix-prefix overlaps between fragments (Sec. III: a fragment is 'fir' when it is a prefix */
/* of another; the weighted overlap graph's edge weights are overlap lengths; Sec. IV: the     */
/* suffix array answers these prefix tests).                                                  */
/* ---------------------------------------------------------------------------------------- */

/* Workspace bytes for sa_overlaps on a text of n bytes with m reads (m <= 0: assume m = n)
 * when the walks find `candidates` suffix/prefix matches (0: the part needed before they are
 * counted). */
int64_t sa_overlaps_ws_bytes(int64_t n, int64_t m, int64_t candidates);

/* sa_overlaps: for every ordered pair of distinct reads (a, b), the largest l with
 * min_len <= l <= min(|a|, |b|) such that the last l bases of a equal the first l bases of b.
 *   sa, isa, lcp  from sa_build / sa_lcp on the same text
 *   out           [cap][3] int32 out: rows (a, b, l) sorted by (a, b), one per pair
 *   n_out_h       host out: number of rows
 *   ws_needed_h   host out, may be NULL: workspace bytes this text needs
 * Returns SA_ERR_NOMEM (with *ws_needed_h set) when ws_bytes is too small -- call again with a
 * larger workspace -- and SA_ERR_CAPACITY (with *n_out_h set) when cap < rows.
 * Synchronises the stream. */
int sa_overlaps(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa,
                const int32_t *lcp, int32_t min_len, int32_t *out, int64_t cap,
                int64_t *n_out_h, void *ws, int64_t ws_bytes, int64_t *ws_needed_h,
                hipStream_t stream);

/* ---------------------------------------------------------------------------------------- */
/* Overlaps on both strands (Sec. III: the second fragment of an overlap may be reversed and   */
/* complemented).  Index the doubled text made by sa_revcomp_text with sa_build / sa_lcp /     */
/* sa_overlaps, then name the rows by strand with sa_strand_rows.                             */
/* ---------------------------------------------------------------------------------------- */

/* sa_revcomp_text: out[0, n) = text; out[n, 2n) = the reverse complement (A<->T, C<->G) of
 * text[0, n-1) followed by '$' -- so read m+k of the doubled text is the reverse complement of
 * read m-1-k.  *m_h = number of reads of text.  out is [2n] device; ws >= 256 bytes.
 * SA_ERR_TOO_LARGE when 2n >= 2^31 - 2.  Synchronises the stream. */
int sa_revcomp_text(const uint8_t *text, int64_t n, uint8_t *out, int64_t *m_h, void *ws,
                    int64_t ws_bytes, hipStream_t stream);

int64_t sa_strand_rows_ws_bytes(int64_t rows, int64_t m);

/* sa_strand_rows: rows [r][3] = sa_overlaps output on a doubled text of 2m reads.  Writes
 * out [cap][4] int32 rows (a, b, strand, l), a != b, sorted by (a, b, strand), naming the
 * original reads a and b and how the overlap of length l joins them:
 *   strand 0: the last l bases of a equal the first l of b;
 *   strand 1: the last l bases of a equal the first l of rc(b)  (their ends meet);
 *   strand 2: the last l bases of rc(a) equal the first l of b  (their starts meet).
 * (rc(a) before rc(b) is b before a, a strand-0 row.)  *n_out_h = number of rows
 * (SA_ERR_CAPACITY when cap is smaller).  SA_ERR_INVALID for a read id >= 2m.  Synchronises
 * the stream. */
int sa_strand_rows(const int32_t *rows, int64_t r, int64_t m, int32_t *out, int64_t cap,
                   int64_t *n_out_h, void *ws, int64_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------- */
/* Assembly-job server: continuous batching of fragment sets (Sec. III: one set of shotgun     */
/* fragments per reconstruction) under an HBM budget.                                         */
/* ---------------------------------------------------------------------------------------- */
typedef struct asm_server asm_server;

typedef struct {
    int32_t status;          /* SA_PENDING, SA_OK or the SA_ERR_* the job failed with */
    int64_t n, m;            /* text length and read count */
    int64_t n_overlaps;      /* rows in ovl */
    const int32_t *sa;       /* [n] device, job-local positions; owned by the server */
    const int32_t *isa;      /* [n] device */
    const int32_t *lcp;      /* [n] device */
    const int32_t *ovl;      /* [n_overlaps][3] device rows (a, b, l), job-local read ids */
    double t_submit, t_admit, t_done;  /* seconds since the server was created */
} asm_result;

/* asm_server_create: start a server over the device buffer `arena` (arena_bytes, the HBM budget;
 * the caller keeps ownership and frees it after asm_server_destroy).
 *   max_jobs_per_batch  upper bound on jobs laid into one batch
 *   workers             worker threads, each with its own HIP stream (1..16); batches on
 *                       different workers run concurrently on the device
 *   mode                0: continuous batching; 1: plain (one job at a time, one worker, the
 *                       single-text entry points) -- the per-job baseline
 * The server uses the device current at creation.  It takes a worker count instead of one
 * caller stream: a batch admitted while another is on the device must run on a stream of its
 * own to overlap with it, so each worker owns one (non-blocking, default priority).  Callers
 * order their own work after a job through asm_poll, which reports a job done only once its
 * results are complete in device memory.
 * Admission: queued jobs are laid into a batch in arrival order, up to max_jobs_per_batch jobs
 * and 2^30 characters, all with the min_len of the first; up to 16 queued jobs that do not
 * match (another min_len, or past the character limit) are passed over and keep their place.
 * The batch is admitted while its memory fits.  When a batch of
 * several jobs does not fit, half as many are tried at once (the full batch size returns with
 * the next admission that fits).  A single job that does not fit waits until a batch ends or
 * the caller releases a finished job (asm_release); it fails with SA_ERR_NOMEM only when it
 * does not fit in an empty arena.  Finished jobs hold their memory until released, so a
 * caller that never releases can leave later jobs waiting. */
int asm_server_create(void *arena, int64_t arena_bytes, int32_t max_jobs_per_batch,
                      int32_t workers, int32_t mode, asm_server **out);

/* asm_submit: queue one job (host text, same conventions as sa_build).
 *   flags 0           the text is validated and copied, so the caller may reuse it at once;
 *                     a bad text returns SA_ERR_ALPHABET / SA_ERR_INVALID here
 *   flags ASM_BORROW  no copy: the caller keeps the text valid and unchanged until asm_poll
 *                     reports a final status; the alphabet is checked by the worker that runs
 *                     the job, and a bad text makes that job (only) finish with SA_ERR_ALPHABET
 * Returns SA_ERR_NOMEM when the job alone exceeds the budget.  The server keeps running after
 * any rejected job. */
enum { ASM_BORROW = 1 };
int asm_submit(asm_server *server, const uint8_t *text_h, int64_t n, int32_t min_len,
               int32_t flags, uint64_t *job_id_h);

/* asm_poll: status and, once done, results of a job.  Returns SA_PENDING while it runs, SA_OK
 * once res_h->status is final (which may itself be an error), SA_ERR_NOTFOUND for an unknown
 * id.  Result pointers stay valid until asm_release. */
int asm_poll(asm_server *server, uint64_t job_id, asm_result *res_h);

/* asm_release: return a finished job's device memory to the arena and forget the job. */
int asm_release(asm_server *server, uint64_t job_id);

/* asm_server_stats: out_h[6] = {batches run, jobs finished, most batches in flight at once,
 * arena bytes in use, arena bytes, jobs queued}. */
int asm_server_stats(asm_server *server, int64_t *out_h);

/* asm_server_fail_alloc_after: make the k-th next arena allocation fail (k >= 1; 0 disarms),
 * to exercise the failure path: the affected batch's jobs fail with SA_ERR_NOMEM, their memory
 * is returned, and other jobs are unaffected. */
int asm_server_fail_alloc_after(asm_server *server, int32_t k);

/* asm_server_destroy: finish queued jobs, stop the workers, free host state. */
int asm_server_destroy(asm_server *server);

/* ---------------------------------------------------------------------------------------- */
/* Measurement support.                                                                      */
/* ---------------------------------------------------------------------------------------- */

/* Per-kernel timing with HIP events recorded on the launch stream around every instrumented
 * launch.  Keys: "radix_pass", "key0" (first-round keys), "keybuild" (doubling keys in text
 * order), "keyruns" (doubling keys sorted run by run), "rank_update", "kasai", "lcp_gather",
 * "overlap_walk", "pack", "lookup".
 * sa_timing_get returns launches, summed duration (ms) and summed algorithmic bytes (the
 * bytes each launch must move at minimum, as documented per kernel). */
int sa_timing_enable(int32_t on);
int sa_timing_reset(void);
int sa_timing_get(const char *key, int64_t *launches_h, double *total_ms_h, double *bytes_h);

/* sa_timing_items: summed units of work of the timed launches under `key` (suffixes for
 * "pack", "key0", "kasai" and "lcp_gather"; items sorted for "radix_pass"; active suffixes
 * for "rank_update", "keyruns" and "keybuild"; reads for
 * "overlap_walk"; patterns for "lookup"), so that bytes per unit of any other model can be
 * applied to the same launches. */
int sa_timing_items(const char *key, double *items_h);

/* sa_copy_u32: plain device copy of n words (dst[i] = src[i]); a reference kernel of known
 * traffic for calibrating hardware byte counters.  Does not synchronise. */
int sa_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SAASM_H */
