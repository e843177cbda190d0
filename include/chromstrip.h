/*
 * chromstrip.h -- C ABI of the MI355X chromatic-strip library.
 *
 * Computes the chromatic polynomial Z = P_G(q) of m x r rectangles of the
 * square or triangular lattice (free boundaries), r = 1..n_max, at integer
 * points q modulo primes p < 2^31, by the sparse transfer-matrix
 * factorisation of J. L. Jacobsen, arXiv 1005.3609:
 *   - Z = <e0| T_last T^{r-1} |e0>                      (Sec. 3, eq. Z_from_T)
 *   - square:     T = T_m ... T_1, T_i = (prod_{j!=i} P_{j,j+1}) V_i H_{i,i+1},
 *                 T_m = (prod_j P_{j,j+1}) V_m          (Sec. 3.2, eqs. T_sq_decomp, T_sq_proj)
 *   - triangular: T_i = P_all V_i H_{i-1,i} H_{i,i+1}   (Sec. 3.3)
 *   - T_last = T_m^last ... T_1^last,
 *     T_i^last = (prod_{j>i} P_{j,j+1}) D_i H_{i,i+1}   (Sec. 3.2, eqs. T_last, T_last_i)
 *   - states: non-crossing non-nearest-neighbour partitions, ranked by the
 *     ordering of Sec. 3.4 (eq. M_recurs); residues mod p < 2^31 (Sec. 3.5).
 * The weights are evaluated at integer q in un-normalised form (a component
 * pays its factor q when it leaves the layer), which equals the paper's
 * normalised P-tilde times q^{|V|} and allows q = 0.
 *
 * Conventions for every call:
 *   - Return value: 0 on success, a negative CHROM_E* code on failure; then
 *     chromatic_last_error() describes it (thread-local, valid until the
 *     next call on the same thread).  No C++ exception crosses this ABI.
 *   - lattice is CHROM_SQUARE or CHROM_TRIANGULAR; 1 <= m <= CHROM_MAX_M;
 *     n_max >= 1 (n_max = 0 is accepted and writes nothing).
 *   - Instances are (q_points[a], primes[b]), a < nq, b < np; results are
 *     laid out out[(r-1)*nq*np + a*np + b] = P_{m x r}(q_a) mod p_b.
 *     Each prime must satisfy 2 < p < 2^31 (not checked for primality);
 *     q is reduced mod p.
 *   - The caller owns every input and output buffer.  The library owns only
 *     its cache of factor maps (host and device copies, per lattice, m and
 *     device), kept until chromatic_release_maps() or process exit.
 *   - Host-pointer arguments are read before the call returns.  Device
 *     pointers must stay valid until the work queued on `stream` finishes.
 *
 * Environment (read when the maps of a (lattice, m) are first built or a
 * job is laid out; none changes any result):
 *   CHROMSTRIP_THREADS=n       host threads for host map builds (default:
 *                              the hardware's count)
 *   CHROMSTRIP_HOST_MAPS=1     build the coefficient form's maps on the host
 *                              and upload them, instead of on the device
 *   CHROMSTRIP_STATE_ORDER=paper  keep the paper's state order between the
 *                              forward factors of host-built maps (default:
 *                              reader order, for locality)
 *   CHROMSTRIP_WIDE_ROWS=1     64-bit row bases in the coefficient form at
 *                              any size (they are used past 4 GiB anyway)
 *   CHROMSTRIP_VERBOSE=1       one stderr line per site of a host map build
 */
#ifndef CHROMSTRIP_H
#define CHROMSTRIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHROM_MAX_M 20

enum {
  CHROM_OK = 0,
  CHROM_EINVAL = -1,        /* bad argument */
  CHROM_ENOMEM = -2,        /* host or device allocation failed / workspace too small */
  CHROM_EDEVICE = -3,       /* a HIP call failed */
  CHROM_EUNSUPPORTED = -4,  /* size or mode the library does not handle */
};

enum { CHROM_SQUARE = 0, CHROM_TRIANGULAR = 1 };

/* Execution modes of chromatic_strip_async. */
enum {
  CHROM_MODE_PLAIN = 0,      /* per-instance vectors [S], one launch per factor per instance */
  CHROM_MODE_BATCHED = 1,    /* instance-minor vectors, one launch per factor for all instances */
  CHROM_MODE_GRAPH = 2,      /* as BATCHED, the rows captured in a hipGraph (up to 32 per graph)
                                and replayed; each chunk group runs its rows as an independent
                                chain */
  CHROM_MODE_RESIDENT = 3,   /* the whole strip in ONE launch: each workgroup keeps the state
                                vectors of lanes_v instances in LDS and runs every factor
                                (Sec. 3.2-3.3) and row read-out (eq. Z_from_T) with workgroup
                                barriers only; for widths whose two vectors fit 160 KiB (square
                                m <= 12, triangular m <= 13 at lanes_v 1), else
                                CHROM_EUNSUPPORTED.  waves_per_block may also be 16. */
  CHROM_MODE_GROUPED = 4,    /* every step one grouped launch; the whole sweep one hipGraph */
};

/* Launch shape of the batched, graph, grouped and resident kernels (and of
 * the coefficient form).  Zero fields take the library's defaults.  Every
 * choice gives bit-identical results. */
typedef struct chrom_tuning {
  int lanes_v;          /* instances per lane: 1, 2 or 4 (chunk width W = 64 * lanes_v);
                           batched and graph modes at 4: when the instance count is not
                           a multiple of 256, the instances past the last multiple run
                           as a second job at 2 (1 for at most 64) beside the first (in
                           graph mode a parallel branch of the same graph) instead of a
                           padded chunk; the coefficient form also takes 8, with unroll
                           4; resident mode: instances per workgroup */
  int targets_per_wave; /* consecutive target states handled by one wavefront, 1..63 */
  int waves_per_block;  /* wavefronts per workgroup: 1, 2, 4 or 8 (resident mode also 16) */
  int xcd_order;        /* 0 = default, 1 = hardware round-robin, 2 = contiguous tile range per XCD,
                           3 / 4 / 5 / 6 = runs of 4 / 16 / 64 / 256 consecutive tiles per
                           XCD, runs round-robin */
  int unroll;           /* source rows loaded ahead per wavefront: 4 or 8 (0 = 4) */
  int streams;          /* instance-chunk groups run on parallel streams, 1..4 (0 = 1);
                           graph and batched modes */
  int fuse;             /* consecutive factors applied per launch as one precomputed
                           product map, 1..3 (0 = 1) */
  int stage;            /* 1: each workgroup first copies the distinct source rows of its
                           tile of consecutive target states into LDS; 2: the same for
                           clustered tiles, targets grouped by the sources they share
                           (chromatic_cluster_export); 3: clustered tiles, each workgroup
                           running a range of them and requesting the next tile's rows
                           while it computes the current one (1-3: batched and graph
                           modes, lanes_v 1 or 2); 4: direct gathers over the clustered
                           order of the targets (no LDS; lanes_v 1, 2 or 4); 5: op-stream gathers, each factor's
                           entries re-encoded as words carrying their coefficient digits
                           and row ends, read through the scalar cache (evaluation form,
                           unit coefficients in powers of t up to t^2 -- the square
                           lattice's single factors and fused pairs -- else CHROM_EINVAL;
                           batched and graph modes, lanes_v 1 or 2, a chunk's vector
                           below 2 GiB); 6: direct gathers over an interleaved order, the
                           k-th row of wavefront w of a workgroup being row k x waves + w
                           of its tile, so the workgroup's wavefronts work on adjacent rows
                           at the same time (batched and graph modes); under 4 and 6 the
                           last factor of a row, which writes the NCNNN states, first takes
                           them in the order of their labels read from point 1 to m; 0:
                           direct gathers.  Grouped launches (grouped strips, chromatic_batch,
                           server steps) take 0, 4 or 6.  Resident mode: 0 = exact double accumulation
                           where every row's sum stays below 2^52 (longest row x max
                           |c(q)| <= 2^21), else modular; 1 = modular arithmetic throughout */
} chrom_tuning;

/* ------------------------------------------------------------------------
 * Whole-strip calls
 * ---------------------------------------------------------------------- */

/* Z_{m x r} = <e0| T_last T^{r-1} |e0> for r = 1..n_max (Sec. 3, eq.
 * Z_from_T; factors of Sec. 3.2-3.3), one instance at a time.  Plain
 * per-instance path, synchronous.  q_points[nq], primes[np] and
 * out[n_max*nq*np] are host memory.  Allocates device memory internally and
 * runs on the null stream of the current device. */
int chromatic_strip(int lattice, int m, int n_max,
                    const uint32_t* q_points, int nq,
                    const uint32_t* primes, int np,
                    uint32_t* out);

/* The same Z_{m x r} (eq. Z_from_T) with all instances in shared launches:
 * each factor T_i (eq. T_sq_decomp; Sec. 3.3) applied to every instance's
 * state vector by one launch per step, residues mod p (Sec. 3.5).  Mode
 * CHROM_MODE_BATCHED, GRAPH, RESIDENT or GROUPED; synchronous, host
 * buffers, internal allocation.  tune may be NULL. */
int chromatic_strip_batched(int lattice, int m, int n_max,
                            const uint32_t* q_points, int nq,
                            const uint32_t* primes, int np,
                            int mode, const chrom_tuning* tune,
                            uint32_t* out);

/* Device-workspace size in bytes needed by chromatic_strip_async for the
 * same arguments: two state vectors over the largest space between factors
 * (NCNNN or square-intermediate states, Sec. 3.4), the read-out vector of
 * eq. T_last, per-instance constants and read-out partials.  It depends on
 * mode and tuning (chunk width, fused products, the grouped mode's stage
 * tables, which grow with n_max).  Returns 0 on bad arguments. */
size_t chromatic_workspace_bytes(int lattice, int m, int n_max, int nq, int np,
                                 int mode, const chrom_tuning* tune);

/* ------------------------------------------------------------------------
 * Coefficient form: the normalised chromatic polynomial of eq. Z_modified,
 * P~ = q^{-|V|} P_G(q), a polynomial in x = 1/q with constant term 1, kept
 * as truncated coefficient arrays mod p (Sec. 3.5: the transfer uses only
 * additions and subtractions; results for several primes combine by CRT).
 * Every state carries, per prime, the coefficients of x^0 .. x^{64 V - 1}
 * (V = tuning lanes_v); the read-out applies T_last to every row's state.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for chromatic_series_async (mode BATCHED or GRAPH).
 * d_max must be below 64 * lanes_v; lanes_v 0 (or tune NULL) takes the
 * smallest of 1, 2, 4, 8 that holds d_max + 1 coefficients, as do
 * chromatic_series_async and chromatic_series.  d_max is at most 511.
 * Returns 0 on bad arguments. */
size_t chromatic_series_workspace_bytes(int lattice, int m, int n_max, int np, int d_max,
                                        int mode, const chrom_tuning* tune);

/* Asynchronous coefficient-form strip.  d_out (device, [n_max][np][d_max+1]
 * uint32): row r, prime b holds the coefficients of x^0 .. x^d_max of
 * P~ for the m x (r+1) rectangle, mod primes[b] (the exact polynomial has
 * degree |V| - 1 = m (r+1) - 1; higher coefficients are 0).  primes: host
 * memory, odd, 2 < p < 2^31.  mode: CHROM_MODE_BATCHED or CHROM_MODE_GRAPH;
 * tune: fuse and stage must be 0 or 1 / 0 (single factors, no staging);
 * lanes_v sets the coefficients kept (64 lanes_v > d_max).  Workspace rules
 * as for chromatic_strip_async. */
int chromatic_series_async(int lattice, int m, int n_max, int d_max,
                           const uint32_t* primes, int np, int mode,
                           const chrom_tuning* tune, void* d_workspace, size_t ws_bytes,
                           void* stream, uint32_t* d_out);

/* Same, synchronous, host output [n_max][np][d_max+1], internal
 * allocation. */
int chromatic_series(int lattice, int m, int n_max, int d_max,
                     const uint32_t* primes, int np, int mode,
                     const chrom_tuning* tune, uint32_t* out);

/* Z_{m x r}, r = 1..n_max (eq. Z_from_T), as chromatic_strip_batched, but
 * queued on `stream` (a hipStream_t; NULL = null stream) with a
 * caller-owned workspace.
 * q_points/primes: host memory, read before return.  d_workspace: device
 * memory of at least chromatic_workspace_bytes(...) bytes, 256-byte
 * aligned, owned by the caller and not used by anything else until the
 * stream has finished.  d_out: device memory [n_max][nq][np].  Builds and
 * uploads the factor maps on first use of (lattice, m) on this device
 * (synchronously).  Returns CHROM_ENOMEM if ws_bytes is too small. */
int chromatic_strip_async(int lattice, int m, int n_max,
                          const uint32_t* q_points, int nq,
                          const uint32_t* primes, int np,
                          int mode, const chrom_tuning* tune,
                          void* d_workspace, size_t ws_bytes,
                          void* stream, uint32_t* d_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * strip as chromatic_strip_async in CHROM_MODE_BATCHED, but with its
 * workspace in a device array the library holds (128 MiB on every GPU it
 * runs on, kept until the process ends).  The call allocates nothing: no
 * hipMalloc, hipFree or pinned staging buffers; the per-instance constants
 * are computed on the device from q_points and primes passed as kernel
 * arguments, so the call only queues kernels on `stream`.
 *   - Before the first call for (lattice, m) on a device, call
 *     chromatic_prepare(lattice, m) (and, for tune->fuse > 1, run
 *     chromatic_strip_async once with that fuse) so the factor maps are on
 *     the device; otherwise CHROM_EINVAL.
 *   - q_points[nq] (nq <= 512), primes[np] (np <= 64): host memory, read
 *     before return.  d_out: device memory [n_max][nq][np], caller-owned.
 *   - tune: streams and stage must be 0 or 1 / 0 (one stream, no staging).
 *   - Returns CHROM_EINVAL if the strip's workspace (what
 *     chromatic_workspace_bytes reports for CHROM_MODE_BATCHED, less its
 *     256-byte graph counter) exceeds 128 MiB: e.g. square m <= 12 at 640
 *     instances, m = 14 at 128.
 *   - Every call on a GPU uses that GPU's one array: calls that overlap on
 *     one GPU (different streams or threads) race and give wrong results.
 *     Nothing carries over from one call to the next (every region the
 *     kernels read is written first in the same call). */
int chromatic_strip_noalloc(int lattice, int m, int n_max,
                            const uint32_t* q_points, int nq,
                            const uint32_t* primes, int np,
                            const chrom_tuning* tune, void* stream, uint32_t* d_out);

/* Measurement hook: queues `rows` rows of the per-site factor kernel
 * (T_1..T_m of eq. T_sq_decomp, read-out fused into T_m) on `stream`, on a
 * workspace that chromatic_strip_async has already run on in
 * CHROM_MODE_BATCHED with the same lattice, m, instances and tuning.  Only
 * the factor launches are queued, so a caller can bracket them with events.
 * The vectors' contents are overwritten (the results are not meaningful). */
int chromatic_factor_launches(int lattice, int m,
                              const uint32_t* q_points, int nq,
                              const uint32_t* primes, int np,
                              int rows, const chrom_tuning* tune,
                              void* d_workspace, size_t ws_bytes, void* stream);

/* Builds (host) and uploads (current device) the factor maps of
 * (lattice, m) ahead of time (the CSR forms of T_i and T_i^last, Sec.
 * 3.2-3.4), so that later calls do no host work. */
int chromatic_prepare(int lattice, int m);

/* Builds the host copy of the factor maps of (lattice, m) only, in the
 * evaluation form (normalised = 0) or the coefficient form (normalised = 1,
 * eq. Z_modified); touches no device.  Host map builds are serialized: one
 * map set builds at a time in the process (each build is itself threaded,
 * CHROMSTRIP_THREADS), and a call for a set already built returns at once.
 * Not supported concurrently with other calls of this library from another
 * host thread: a run that did so once crashed in the caller's interpreter
 * and the cause was not found, so call it from the thread that makes the
 * library's other calls.  Returns 0 or CHROM_EINVAL. */
int chromatic_prepare_host(int lattice, int m, int normalised);

/* Builds the coefficient form's factor maps of (lattice, m) on the current
 * device (or on the host and uploads them, with CHROMSTRIP_HOST_MAPS=1)
 * ahead of time.  The first coefficient-form call for (lattice, m) does this
 * itself, with allocations and synchronous copies, so call this first when
 * that call is to be captured in a hipGraph.  Returns 0 or a CHROM_E* code. */
int chromatic_prepare_series(int lattice, int m);

/* Copies one coefficient-form factor map of (lattice, m) as the current
 * device holds it (built there, or uploaded with CHROMSTRIP_HOST_MAPS=1) to
 * the host: which = 4 forward factor T_{idx+1}, 5 read-out factor
 * T_{idx+1}^last, both in gather form.  Call once with null row_ptr and
 * entries for the sizes, then with host buffers of n_rows + 1 and nnz
 * words.  Entry layout as the kernels read it: source rank in bits 0-25,
 * coefficient code in bits 26-31 (codes as chromatic_code_table with
 * normalised = 1).  Returns 0 or a CHROM_E* code. */
int chromatic_series_map_export(int lattice, int m, int which, int idx, int64_t* n_rows, int64_t* n_cols,
                                int64_t* nnz, int32_t* row_ptr, uint32_t* entries);

/* Host-side check of the per-state expansion that builds the coefficient
 * form's maps on the device (Sec. 3.1-3.4): the same expansion and CSR
 * assembly run on the host and are compared, factor by factor, with the
 * host builder's maps of (lattice, m) in the paper's state order (every
 * forward factor; with normalised = 1 also every read-out factor).  Touches
 * no device.  Returns 0 when identical, CHROM_EUNSUPPORTED with the first
 * difference as the error message otherwise. */
int chromatic_check_expansion(int lattice, int m, int normalised);

/* Frees every cached map on host and devices.  Must not run concurrently
 * with any other call of the library. */
void chromatic_release_maps(void);

/* ------------------------------------------------------------------------
 * Many strips of uneven size in shared grouped launches
 * ---------------------------------------------------------------------- */
typedef struct chrom_job {
  int lattice;
  int m;
  int n_max;
  const uint32_t* q_points;  /* host, nq entries */
  int nq;
  const uint32_t* primes;    /* host, np entries */
  int np;
  uint32_t* d_out;           /* device, [n_max][nq][np] */
} chrom_job;

/* Workspace bytes for chromatic_batch over these jobs (each job's vectors
 * as for chromatic_workspace_bytes, plus the stage tables of the grouped
 * launches). */
size_t chromatic_batch_workspace_bytes(const chrom_job* jobs, int njobs,
                                       const chrom_tuning* tune);

/* Z_{m x r} of every job (eq. Z_from_T, factors of Sec. 3.2-3.3, residues
 * of Sec. 3.5), to completion on `stream` as ONE hipGraph launch: each job
 * is split into instance chunks of width 64*lanes_v, and step k of every
 * (job, chunk) item runs in one grouped kernel launch whose workgroups map
 * to (item, tile) pairs, so jobs of uneven state-space size share every
 * launch.  tune->streams is ignored (one launch chain); tune->stage must
 * be 0, 4 or 6 (the grouped kernel gathers directly; 4 and 6 reorder each
 * factor's targets as for a strip), else CHROM_EINVAL.  The graph is
 * captured once per workspace and job list and replayed on later identical
 * calls.  Same results as chromatic_strip for each job.  The workspace must
 * not be reused for another job list while a launch on it is in flight, and
 * its size (chromatic_batch_workspace_bytes) depends on the tuning. */
int chromatic_batch(const chrom_job* jobs, int njobs, const chrom_tuning* tune,
                    void* d_workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Continuous-batching server step
 * ---------------------------------------------------------------------- */
typedef struct chrom_slot {
  int lattice;
  int m;
  int n_max;
  int rows_done;             /* in: rows already read out (0 for a new job); out: updated */
  int nq, np;
  const uint32_t* q_points;  /* host (read only when rows_done == 0) */
  const uint32_t* primes;    /* host (read only when rows_done == 0) */
  void* d_state;             /* device, chromatic_slot_state_bytes(...) bytes, kept between steps */
  size_t state_bytes;
  uint32_t* d_out;           /* device, [n_max][nq][np] */
} chrom_slot;

/* Device bytes a job keeps resident between server steps (two state
 * vectors over the spaces of Sec. 3.4, the read-out vector of eq. T_last,
 * coefficient tables, scratch). */
size_t chromatic_slot_state_bytes(int lattice, int m, int nq, int np,
                                  const chrom_tuning* tune);

/* Continuous batching of strips: the next rows of each slot's Z_{m x r}
 * (one application of T = T_m ... T_1 and one read-out per row, eqs.
 * T_sq_decomp, Z_from_T).  Advances every slot by up to `rows` rows (a new
 * slot first runs its
 * set-up and reads out r = 1) on `stream`, and updates rows_done.  Step k of
 * every slot runs in one grouped launch, so slots that differ in lattice, m
 * and instance count share each launch.  tune->stage: 0, 4 or 6 as for
 * chromatic_batch (the vectors keep their layout, so steps may differ).
 * Server steps on
 * one device must be issued on one stream (they share a stage-table
 * buffer). */
int chromatic_server_step(chrom_slot* slots, int nslots, int rows,
                          const chrom_tuning* tune, void* stream);

/* Synchronises `stream` and reports a pending HIP error (CHROM_EDEVICE). */
int chromatic_device_status(void* stream);

/* ------------------------------------------------------------------------
 * Host-side introspection (no GPU needed): states and factor maps
 * ---------------------------------------------------------------------- */

/* Motzkin number M_k (eq. M_recurs), 0 <= k <= 40; -1 if out of range. */
int64_t chromatic_motzkin(int k);

/* Spaces: CHROM_SPACE_NCNNN (i ignored), CHROM_SPACE_SQ_INTER (square
 * states after T_i, 1 <= i < m: NCNNN plus i~i+1, Sec. 3.4 last paragraph),
 * CHROM_SPACE_LAST (states after T_i^last, 0 <= i <= m: points 1..i
 * singletons, the rest NCNNN). */
enum { CHROM_SPACE_NCNNN = 0, CHROM_SPACE_SQ_INTER = 1, CHROM_SPACE_LAST = 2 };

/* Number of states of a space; < 0 on bad arguments. */
int64_t chromatic_space_size(int m, int space, int i);

/* Rank (0-based, in the paper's order) of the partition given by block
 * labels lab[m] (any labelling; equal labels = same block).  Returns -1 if
 * the partition is not in the space, < -1 on bad arguments. */
int64_t chromatic_rank(int m, int space, int i, const uint8_t* lab);

/* Writes the canonical block labels (first-appearance numbering) of the
 * state of rank r into lab[m]. */
int chromatic_unrank(int m, int space, int i, int64_t r, uint8_t* lab);

/* Summary of the single-factor maps of (lattice, m), building them if
 * needed. */
typedef struct chrom_maps_info {
  int n_factors;            /* m forward factors T_1..T_m */
  int n_last;               /* m read-out factors (T_1^last..T_m^last, transposed) */
  int n_codes;              /* coefficient codes of the single factors */
  int64_t total_nnz;
  int64_t max_states;
} chrom_maps_info;

int chromatic_maps_info(int lattice, int m, chrom_maps_info* info);

/* Factor family `fuse` (1 = the single factors T_1..T_m; k = 2, 3 = the
 * products T_hi ... T_lo of k consecutive factors, lo = idx*k + 1,
 * hi = min(m, lo + k - 1), used by tuning.fuse = k): number of factors and
 * the coefficient table.  coef (may be NULL) receives n_codes x 4 int64
 * values: code c means coef[4c] + coef[4c+1] q + coef[4c+2] q^2 + coef[4c+3] q^3.
 * The table extends the single factors' table, code numbers unchanged. */
int chromatic_family_info(int lattice, int m, int fuse, int* n_factors, int* n_codes, int64_t* coef);

/* Copies one factor's map to caller buffers.  which = 0: forward factor
 * T_{idx+1} as target-major CSR (rows = states after the factor, entries =
 * source states before it).  which = 1: read-out factor T_{idx+1}^last,
 * transposed (rows = states before it, entries = states after it).
 * which = 2 or 3: factor idx of the fused family of that size.
 * which = 4: forward factor T_{idx+1} of the normalised (coefficient-form)
 * set; which = 5: its read-out factor T_{idx+1}^last in gather form (rows =
 * states after it, entries = states before it).  Codes index
 * chromatic_code_table of the same form.
 * Entry word: bits 0..25 = column state rank, bits 26..31 = coefficient
 * code.  Sizes are returned through n_rows, n_cols, nnz; pass NULL buffers
 * to query sizes only.  row_ptr has n_rows+1 entries.  The state numbering
 * of the spaces between factors is internal (chosen for memory locality);
 * the NCNNN space before the first and after the last factor of a row, and
 * the read-out spaces, use the paper's order. */
int chromatic_map_export(int lattice, int m, int which, int idx,
                         int64_t* n_rows, int64_t* n_cols, int64_t* nnz,
                         int32_t* row_ptr, uint32_t* entries);

/* Coefficient table of the maps of (lattice, m): code c is the polynomial
 * coef[4c] + coef[4c+1] z + coef[4c+2] z^2 + coef[4c+3] z^3 with z = q
 * (normalised = 0, the evaluation form) or z = x = 1/q (normalised = 1, the
 * coefficient form).  Pass coef = NULL to query n_codes. */
int chromatic_code_table(int lattice, int m, int normalised, int* n_codes, int64_t* coef);

/* The staged-tile form (tuning field `stage`) of forward factor idx of the
 * fuse-sized family, for a given slot limit and rows-per-tile limit: tiles of
 * consecutive target rows (tile t = rows tile_row0[t] .. tile_row0[t+1]-1,
 * n_tiles + 1 entries), each with its distinct source states
 * src[tile_src0[t] .. tile_src0[t+1]) in ascending order (n_src in all), and
 * the entry words of the factor's CSR (same order, same row pointers as
 * chromatic_map_export) with the source replaced by its slot in the tile's
 * list.  A tile grows row by row while it has at most `rows` rows and
 * `slots` sources; a single row with more sources forms a tile of its own;
 * max_slots is the largest list.  Host-only (no device work).  Pass NULL
 * buffers to query sizes; entries has the factor's nnz words. */
int chromatic_stage_export(int lattice, int m, int fuse, int idx, int slots, int rows,
                           int32_t* n_tiles, int64_t* n_src, int32_t* max_slots,
                           int32_t* tile_row0, int32_t* tile_src0, int32_t* src,
                           uint32_t* entries);

/* The op-stream form (tuning `stage` = 5) of forward factor idx of the
 * fuse-sized family, evaluation form: the basis shift s of the family's
 * kernels, and one word per entry in target row order -- bits 0..22 the
 * source state, bits 24 + 2k / 25 + 2k set for a digit d_k = +1 / -1 of the
 * entry's coefficient in powers of t = q - s (k = 0..2), bit 31 on the last
 * word of a row; a row without entries is one word with only bit 31 -- then
 * 64 zero words.  row_first[r] (n_rows + 1 entries) is the first word of row
 * r.  CHROM_EINVAL when a code has a digit outside -1..1 or a t^3 term.
 * Host-only.  Pass NULL buffers to query n_words (the padding included). */
int chromatic_op_export(int lattice, int m, int fuse, int idx, int32_t* shift, int64_t* n_words,
                        int32_t* row_first, uint32_t* words);

/* The clustered staged-tile form (tuning `stage` = 2) of forward factor idx
 * of the fuse-sized family: tiles of target rows that read the same sources.
 * A tile grows from the lowest unplaced target by adding every unplaced
 * reader of the sources it already reads, while it keeps at most `rows`
 * targets and `slots` distinct sources; when that closes, the next unplaced
 * target seeds it again if it fits (a single row with more sources forms a
 * tile of its own).  Tile t holds positions tile_row0[t] .. tile_row0[t+1]-1
 * (n_tiles + 1 entries); position k writes target row tgt[k] and has the
 * entries row_ptr[k] .. row_ptr[k+1]-1 of `entries` (the factor's entry
 * words with the source replaced by its slot in the tile's list
 * src[tile_src0[t] .. tile_src0[t+1]), ascending).  tgt and row_ptr have
 * n_rows and n_rows + 1 entries, entries the factor's nnz.  Host-only (no
 * device work).  Pass NULL buffers to query sizes. */
int chromatic_cluster_export(int lattice, int m, int fuse, int idx, int slots, int rows,
                             int32_t* n_tiles, int64_t* n_src, int32_t* max_slots,
                             int32_t* tile_row0, int32_t* tile_src0, int32_t* src,
                             int32_t* tgt, int32_t* row_ptr, uint32_t* entries);

/* Thread-local description of the last error. */
const char* chromatic_last_error(void);

/* Library version string. */
const char* chromatic_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CHROMSTRIP_H */
