/*
 * srla.h -- C ABI of the MI355X (gfx950) SRLA library.
 *
 * SRLA (arXiv 1803.10369) detects super points -- hosts of network A that
 * talk to at least theta distinct hosts of network B inside a sliding window
 * of k time slices (Section 3.1, Definitions 1-2) -- and estimates their
 * cardinality.  Every (aip, bip) pair of a slice (Definition "IPpair",
 * Section 3.2) is scanned into an array of sliding estimators (the SEA of
 * Section 4.1: u rows of SE, each SE holding a sliding rough estimator SRE
 * of g distance recorders, a 16-bit super point indicator SI, and a linear
 * estimator LE of g' distance recorders).  At the end of every slice the
 * candidate list is finished, every candidate's cardinality is estimated
 * with the noise-corrected union estimate (Eq8-Eq9, Section 4.2), and the
 * array is prepared for the next slice (Algorithm 3).
 *
 * Every function returns an int status (SRLA_OK or a negative SRLA_E_*) and
 * never throws.  A monitor is not thread-safe; separate monitors are
 * independent.  Scans run on the monitor's scan stream (the caller's, or one
 * the library creates); the end-of-slice work runs on a second stream the
 * library owns, ordered after the slice's scans by HIP events, so that the
 * next slice can be scanned while the previous one is being estimated.
 */
#ifndef SRLA_H
#define SRLA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SRLA_OK = 0,
    SRLA_E_INVAL = -1,     /* bad argument; nothing was changed */
    SRLA_E_NOMEM = -2,     /* a device or pinned host allocation failed */
    SRLA_E_CAPACITY = -3,  /* the candidate list outgrew max_candidates */
    SRLA_E_STATE = -4,     /* the monitor is poisoned by an earlier error */
    SRLA_E_DEVICE = -5     /* a HIP runtime call failed */
};

/* srla_dump_state: which array */
enum { SRLA_DUMP_LE = 0, SRLA_DUMP_RE = 1, SRLA_DUMP_SI = 2 };

/* per-candidate report flags */
enum {
    SRLA_FLAG_SUPER = 1,  /* estimate >= threshold: a detected super point */
    SRLA_FLAG_SAT = 2,    /* Eq9 undefined (union LE full); estimate is +inf */
    SRLA_FLAG_NEW = 4,    /* inserted into the candidate list in this slice */
    SRLA_FLAG_KEEP = 8    /* carried into the next slice by Algorithm 3 */
};

/* srla_config_t.flags */
enum {
    SRLA_CFG_TIMING = 1,   /* record HIP events around every stage */
    SRLA_CFG_SCAN_XCD = 2, /* scan with per-XCD row ownership (each XCD stores
                              into its own SEA rows); results are identical
                              either way, only the speed differs */
    SRLA_CFG_GRAPH = 4,    /* record the end-of-slice pipeline once per slice
                              parity as HIP graphs and replay them; results
                              are identical either way.  Graphs save the host
                              the launches; on the device each graph launch
                              leaves a gap of 10-20 us, which kernels
                              launched one by one on the same stream do not,
                              so with SRLA_CFG_HOLD_SCANS (the slice end on
                              the scan stream) launching kernel by kernel was
                              faster (16.5 against 16.0 G packets/s) */
    SRLA_CFG_DISCRETE = 8, /* the discrete-window form (Section 3.2: with
                              k = 1 a one-bit DR suffices; Section 5.1 runs
                              it with z = 1): every DR is one bit, set by the
                              scan and cleared at the slice's end.  Requires
                              window_slices == 1; reports are identical to
                              the 16-bit form's at k = 1.  SRLA_CFG_SCAN_XCD
                              has no effect; such monitors cannot join a
                              group */
    SRLA_CFG_LEAN_REPORT = 16, /* reports carry ip, est and flags only
                                  (union_weight and re_weight are NULL):
                                  13 instead of 18 bytes per candidate cross
                                  PCIe at every slice end */
    SRLA_CFG_SCAN_DEDUP = 32,  /* scan in read-before-write form: a DR that
                                  already holds the open slice's stamp is not
                                  stored again (DRset is idempotent).  Results
                                  are identical; faster when pairs repeat DRs
                                  often.  With SRLA_CFG_SCAN_XCD as well, each
                                  XCD reads and stamps only its own rows
                                  (u in {1, 2, 4, 8, 16} and 16-byte aligned
                                  device pairs; otherwise the flat
                                  read-before-write form) */
    SRLA_CFG_SCAN_LDS_FILTER = 64, /* scan with a workgroup filter of repeated
                                  stores: each workgroup keeps the LE DRs it
                                  stored last in an LDS table and skips
                                  stores it has already issued in this scan.
                                  Results are identical.  Below
                                  SRLA_CFG_SCAN_DEDUP, above
                                  SRLA_CFG_SCAN_XCD in precedence */
    SRLA_CFG_OVERLAP_REPORT = 128 /* for the streaming form: the candidate
                                  check and the estimate of a closed slice
                                  run before the next slice's scans may start
                                  (into device staging arrays), and only the
                                  PCIe copy of the report runs alongside
                                  those scans -- enqueued by the next slice's
                                  first srla_scan, after that scan has
                                  started, or by srla_wait_report if it comes
                                  first.  Results are identical; costs two
                                  staging sets (by slice parity) of 13
                                  (lean) or 18 bytes of device memory per
                                  max_candidates.  Such monitors cannot join
                                  a group */,
    SRLA_CFG_SCAN_PARTITION = 256 /* scan in partitioned form: each chunk of
                                  pairs sorts its LE DR indices by region
                                  of 2^16 DRs, then workgroups (units of
                                  about 32768 indices of one region) mark
                                  the DRs named in them and one workgroup
                                  per half region stamps them, so the LE
                                  stores fill whole cache lines instead of
                                  going out one 2-byte store at a time.
                                  Results are identical.  Any LE: one of
                                  more than 2^27 DRs (u * v_le * g_le) is
                                  taken in bands of 2^27 DRs, one read of
                                  the pairs per band.  Costs 128 MiB of
                                  device scratch plus, for R = min(regions,
                                  2048), 4 KiB * (R + 1) (offsets) and 8 KiB
                                  * (R + 2048) (unit bitmaps): at most 168
                                  MiB.  Above every other scan form in
                                  precedence; no effect in the discrete
                                  form.  A group whose members all have it
                                  runs each member's partitioned scan over
                                  the pairs instead of the fused kernel */,
    SRLA_CFG_HOLD_SCANS = 1024 /* for the streaming form: scans issued after
                                  srla_close_slice of slice e start on the
                                  device only once e's report is in host
                                  memory, so e's end-of-slice work runs
                                  without a scan beside it (the scans
                                  overlap only Algorithm 3's carried list
                                  and SI update, which the report does not
                                  wait for).  The sort, the candidate check,
                                  the estimate and the report then run on
                                  the monitor's (scan) stream, in order
                                  after the scans, and the next scans
                                  follow them there.  The host can still
                                  close e and issue e+1's scans at once, so
                                  no host round trip separates a slice's
                                  scans from its end-of-slice work.
                                  Results are identical; no effect with
                                  SRLA_CFG_OVERLAP_REPORT */
};

/*
 * SEA geometry (Section 4.1).  Row i of the array holds v_re SEs worth of SI
 * and SRE and v_le SEs worth of LE; the paper's SE is v_re == v_le.  The
 * distance recorders are z = 16 bits wide (Section 3.2).
 *   u        rows, 1..16 (the paper uses 4)
 *   v_re     SI/SRE columns per row, >= 1
 *   g        DRs per SRE, 1..64 (the paper: 8 is enough for IPv4)
 *   v_le     LE columns per row, >= 1
 *   g_le     DRs per LE (the paper's g'), a positive multiple of 64
 *   hash_seed  seed of every hash function of the monitor
 */
typedef struct {
    uint32_t u, v_re, g, v_le, g_le;
    uint64_t hash_seed;
} srla_geometry_t;

/*
 *   window_slices   k, the sliding window W(t, k) in slices, 1..32767
 *                   (Section 3.1; a 16-bit DR allows k < 2^16, and the
 *                   library keeps half of that range as aging slack)
 *   threshold       theta >= 1 (Definition 2)
 *   max_candidates  capacity of the candidate list, >= 1
 *   flags           SRLA_CFG_* bits
 *   scan_blocks     launch-shape knob of the scan kernel: the most
 *                   workgroups one scan launch uses (they stride over the
 *                   pairs); 0 = one workgroup per tile of 2048 pairs.  With
 *                   SRLA_CFG_SCAN_PARTITION: the DR indices per marking unit
 *                   (a power of two from 8192 to 131072; 0 = 32768), whose
 *                   bitmaps (8 KiB each, at most R + 2^26 / unit of them)
 *                   count in the scratch.  Results do not depend on it.
 */
typedef struct {
    uint32_t window_slices;
    uint32_t threshold;
    srla_geometry_t geom;
    uint64_t max_candidates;
    uint32_t flags;
    uint32_t scan_blocks;
} srla_config_t;

typedef struct srla_monitor srla_monitor_t;

/*
 * The report of one closed slice e, covering the window [e-k+1, e]
 * (window_full == 0 while e < k-1).  Arrays are pinned host memory owned by
 * the library, written by its kernels (three sets, used by slices in turn);
 * they stay valid until slice e+2 is closed (srla_close_slice or
 * srla_estimate) or srla_destroy.  They are read-only for the caller: the
 * library keeps a device copy of what each set's est and flags hold and
 * writes only the entries that change (except with SRLA_CFG_OVERLAP_REPORT).
 *   ip            the candidate list CSIP = NCSIP + N (Algorithms 2-3): the
 *                 candidates carried from slice e-1, ascending, then the new
 *                 candidates of slice e (flag NEW), ascending
 *   est           Eq9 estimate of |OP(ip, e-k+1, k)| (FP64; +inf with SAT)
 *   flags         SRLA_FLAG_* of each candidate
 *   union_weight  |ULE(ip)|^k, union LE DRs inside the window (Algorithm 1)
 *   re_weight     |URE(ip)|^k before the slide
 *                 (both NULL with SRLA_CFG_LEAN_REPORT)
 *   row_fill      |LDR(i)|^k for i < u: LE DRs of row i inside the window
 *   up            Eq8
 *   n_touched     distinct sources with at least one SRE-sampled pair in e
 *   n_new         candidates inserted in e
 *   latency_ms    device time from the end of e's last scan (for a slice
 *                 without scans: the start of its end-of-slice work) until
 *                 the report was complete in host memory (device wall clock)
 *   host_bytes    bytes e's end-of-slice work wrote into the report arrays
 *                 (est and flags pieces that changed, the new candidates'
 *                 addresses, union_weight and re_weight; the carried
 *                 candidates' addresses go in beside the scans and are not
 *                 counted); with SRLA_CFG_OVERLAP_REPORT the staged bytes
 */
typedef struct {
    uint64_t slice;
    uint32_t window_full;
    uint64_t n;
    const uint32_t *ip;
    const double *est;
    const uint8_t *flags;
    const uint32_t *union_weight;
    const uint8_t *re_weight;
    const uint64_t *row_fill;
    double up;
    uint64_t n_touched;
    uint64_t n_new;
    double latency_ms;
    uint64_t host_bytes;
} srla_report_t;

/* Accumulated stage times (milliseconds, HIP events on the stream each stage
   runs on) since the last reset; all zero unless SRLA_CFG_TIMING was set (or
   timing was switched on with srla_set_timing).  scan_launches and
   scan_pairs count the scans whose time is included in scan_ms (fused group
   scans are counted but not timed), estimates the closed slices whose
   end-of-slice stages are included.
   With SRLA_CFG_GRAPH each of the two end-of-slice phases is timed as one:
   the sweeps (sweep_ms, or estimate_ms together with the candidate work when
   SRLA_CFG_OVERLAP_REPORT moves it there) and the rest (estimate_ms, or
   report_ms for the overlapped report copy). */
typedef struct {
    double scan_ms;        /* Algorithm 2 scan kernels */
    uint64_t scan_launches;
    uint64_t scan_pairs;
    double sweep_ms;       /* row fills |LDR(i)|^k and the LE/SRE activity bitmaps */
    double finalize_ms;    /* candidate check of the slice's sampled sources */
    double estimate_ms;    /* merge, Eq8-Eq9 and the Algorithm 3 re-check */
    double slide_ms;       /* carried-list compaction, SI update, status */
    double report_ms;      /* report copy to the host (SRLA_CFG_OVERLAP_REPORT) and
                              the status block */
    uint64_t estimates;
} srla_timings_t;

/*
 * Device bytes a monitor of this configuration allocates (DR arrays, SI
 * counters, activity bitmaps, candidate buffers; the slice's sampled-source
 * list grows with the pairs scanned and is not included).  0 for an invalid
 * config.
 */
uint64_t srla_footprint_bytes(const srla_config_t *cfg);

/*
 * Admission of monitors by device footprint: walks cfgs[0..n) in order and
 * admits each one whose srla_footprint_bytes still fits in what remains of
 * budget_bytes (first fit; a rejected monitor does not stop later, smaller
 * ones).  admitted[i] is set to 1 or 0; *used_bytes to the admitted total.
 * Host-only.  Errors: SRLA_E_INVAL (NULL arrays, an invalid config).
 */
int srla_admit(const srla_config_t *cfgs, uint32_t n, uint64_t budget_bytes, uint8_t *admitted,
               uint64_t *used_bytes);

/*
 * Creates a monitor on the current HIP device.  hip_stream is a hipStream_t
 * on which every operation of the monitor is issued; NULL makes the library
 * create (and later destroy) its own stream.  All DRs start as DRinit (never
 * set), all SI bits as 0, the open slice is 0.  *out is set only on success.
 * Errors: SRLA_E_INVAL (cfg out of range, NULL out), SRLA_E_NOMEM,
 * SRLA_E_DEVICE.
 */
int srla_create(const srla_config_t *cfg, void *hip_stream, srla_monitor_t **out);

/*
 * Scans n pairs into the open slice (Algorithm 2, Section 4.1): every pair
 * sets one LE DR in each row; pairs whose bip hashes to LSB(H1(bip)) >= tau
 * (Eq1) also set one SRE DR per row and mark aip as sampled in this slice.
 * pairs: 2n uint32 values, interleaved (aip, bip), host byte order.
 * on_device != 0: pairs is device memory readable on the monitor's stream;
 *   the caller keeps it alive until the work has run (the next
 *   srla_estimate returns after it).
 * on_device == 0: pairs is host memory, copied before this call returns:
 *   in chunks of 4M pairs by DMA on a library stream, overlapping the scans
 *   of earlier chunks; page-locked memory (hipHostMalloc, torch pin_memory)
 *   is read by the DMA directly, pageable memory through two pinned
 *   bounce buffers.
 * May be called any number of times per slice; the order of pairs does not
 * change any result.  Errors: SRLA_E_INVAL (NULL pairs with n > 0),
 * SRLA_E_STATE (poisoned), SRLA_E_NOMEM, SRLA_E_DEVICE.
 */
int srla_scan(srla_monitor_t *m, const uint32_t *pairs, uint64_t n, int on_device);
/* (In the discrete form the SRE and LE of the open slice are fresh bit
   arrays; the scan ORs bits into them, and sampled sources go into the
   slice's source set.) */

/*
 * srla_scan without allocation, for callers that cannot allocate device
 * memory (code under HIP stream capture, serving loops that forbid
 * hipMalloc): the same scan (results identical to srla_scan's), always in
 * the partitioned form, with its scratch -- DR-index blocks, region offsets,
 * marking bitmaps -- in one fixed library array of 24.5 MiB per device
 * (allocated when the library is loaded, held until the process ends)
 * instead of memory the call or the monitor allocates.  It calls no
 * allocator, grows no buffer and records no timing events.
 * pairs: 2n uint32 values (aip, bip) in device memory readable on the
 *   monitor's stream, kept alive until the scan has run.
 * Limits (violations return SRLA_E_INVAL and change nothing): the slice's
 *   pairs so far plus n within the sampled-source capacity the monitor
 *   holds (2^20 pairs at creation; srla_scan grows it to the largest slice
 *   it has scanned); any LE size (bands of 2^26 DRs as above); not for
 *   SRLA_CFG_DISCRETE or SRLA_CFG_OVERLAP_REPORT monitors.
 * All monitors on a device share its one scratch array and every call
 * leaves its own contents there: scans that overlap in time on one device
 * (monitors on different streams) race and must be ordered by the caller.
 * Errors: SRLA_E_INVAL, SRLA_E_STATE (poisoned), SRLA_E_DEVICE.
 */
int srla_scan_noalloc(srla_monitor_t *m, const uint32_t *pairs, uint64_t n);

/*
 * Closes the open slice e and fills *out with its report (Section 4.2 and
 * Algorithm 3): the candidate check of every source sampled in e against the
 * union SRE and union SI, the union-LE estimate (Eq8-Eq9) of every candidate,
 * then the slide -- SI cleared, every DR one slice older, candidates whose
 * union SRE still passes carried into slice e+1 with their SI bits set.
 * Blocks until the report is in host memory.  Same as srla_close_slice
 * followed by srla_wait_report.  Errors: SRLA_E_CAPACITY (more than
 * max_candidates candidates; the monitor is then poisoned), SRLA_E_STATE
 * (poisoned, or an earlier closed slice's report not collected),
 * SRLA_E_INVAL (NULL out), SRLA_E_NOMEM, SRLA_E_DEVICE.
 */
int srla_estimate(srla_monitor_t *m, srla_report_t *out);

/*
 * Streaming form of srla_estimate.  srla_close_slice closes the open slice e
 * without waiting: it enqueues e's end-of-slice work and opens slice e+1 at
 * once.  Scans of e+1 may be issued right away; on the device they start as
 * soon as e's DRs have been snapshotted (the LE/SRE activity sweeps, which
 * run on the monitor's stream right after e's scans), and run while e is
 * still being estimated.  srla_wait_report blocks until the report of the
 * oldest closed slice not yet collected is in host memory and fills *out.
 * At most two closed slices may wait for collection: e+1 may be closed before
 * e's report is collected, so the caller can issue a slice's close ahead of
 * waiting for the previous report; a third close returns SRLA_E_STATE.
 * srla_estimate requires that no report is waiting.  Results are identical
 * to srla_estimate's.  Errors as for srla_estimate; SRLA_E_CAPACITY is
 * reported by srla_wait_report.
 */
int srla_close_slice(srla_monitor_t *m);
int srla_wait_report(srla_monitor_t *m, srla_report_t *out);

/*
 * Copies one state array to host memory, as of the open slice.
 * which = SRLA_DUMP_LE: u*v_le*g_le values, layout [row][column][DR];
 *         SRLA_DUMP_RE: u*v_re*g values, layout [row][column][DR];
 *   each value is the DR's distance in slices (Section 3.2), with distances
 *   of 32768 and more (and never-set DRs) written as 65535.
 * which = SRLA_DUMP_SI: u*v_re raw 16-bit SI words, layout [row][column].
 * In the discrete form a DR is one bit and its distance is written as 0
 * (set in the open slice), 1 (set only in the slice closed last) or 65535.
 * cells must equal the array's size.  Blocks until the copy is done.
 */
int srla_dump_state(srla_monitor_t *m, int which, uint16_t *host_out, uint64_t cells);

/* Stage times since the last reset (reset != 0 clears them after reading). */
int srla_timings(srla_monitor_t *m, srla_timings_t *out, int reset);

/*
 * Switches the per-stage timing on (enabled != 0) or off for the calls that
 * follow: scans issued and slices closed while it is on are timed (a closed
 * slice's stages are timed as it was when it was closed).  Each timed stage
 * costs two HIP event records on its stream, and a record costs the stream
 * some microseconds (a backbone slice: 14.4 G packets/s with every stage
 * timed, 15.6 G untimed), so a caller that needs the times but not for every
 * slice can time a sample of the slices.  enabled == SRLA_TIMING_SCANS times
 * the scans only (scan_ms, scan_launches, scan_pairs).  Totals are kept
 * across switches.  Errors: SRLA_E_INVAL (NULL monitor).
 */
#define SRLA_TIMING_SCANS 2
int srla_set_timing(srla_monitor_t *m, int enabled);

/*
 * Monitor groups: many monitors -- each with its own window, DR geometry,
 * threshold and hash seed -- fed the same pair stream.  srla_group_scan runs
 * one fused scan kernel that loads every pair once and applies Algorithm 2
 * of every member (or, when every member has SRLA_CFG_SCAN_PARTITION,
 * each member's partitioned scan in turn); it is equivalent to srla_scan on
 * each member with the same pairs.  Slices are still closed and reported per member
 * (srla_close_slice / srla_wait_report / srla_estimate).
 * srla_group_create: 1..64 distinct monitors that share one scan stream,
 *   none of them in the discrete form or with SRLA_CFG_OVERLAP_REPORT;
 *   scan_blocks as in srla_config_t.  The group does not own the monitors;
 *   destroy the group before any member.
 * srla_group_scan: pairs as for srla_scan, device memory only (on_device
 *   must be nonzero).  Errors: SRLA_E_INVAL, SRLA_E_STATE (a member is
 *   poisoned), SRLA_E_NOMEM, SRLA_E_DEVICE.
 */
typedef struct srla_group srla_group_t;
int srla_group_create(srla_monitor_t *const *monitors, uint32_t n, uint32_t scan_blocks,
                      srla_group_t **out);
int srla_group_scan(srla_group_t *g, const uint32_t *pairs, uint64_t n, int on_device);
int srla_group_destroy(srla_group_t *g);
const char *srla_group_last_error(const srla_group_t *g);

/* Waits for the monitor's streams and frees everything it owns. NULL is ok. */
int srla_destroy(srla_monitor_t *m);

/* Text of the monitor's last error ("" if none); static text for NULL. */
const char *srla_last_error(const srla_monitor_t *m);

#ifdef __cplusplus
}
#endif

#endif /* SRLA_H */
