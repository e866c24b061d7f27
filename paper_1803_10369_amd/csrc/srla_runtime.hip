// Host runtime of the gfx950 SRLA library: the C ABI of include/srla.h.
//
// One monitor = one SEA (Section 4.1) resident in device memory plus the
// buffers of the end-of-slice pipeline.  srla_scan enqueues Algorithm 2 on
// the scan stream (the caller's), in the form the config picks (flat,
// per-XCD, read-before-write, LDS-filtered, or the one-bit discrete form);
// host pairs reach the device by DMA on a third, library-owned stream.
// srla_close_slice enqueues, on the library's pipeline stream, after the
// slice's last scan:
//   snapshot -> |LDR(i)|^k, the LE activity bitmap, the SRE activity map
//               (the end-of-slice state of every DR; scans of the next slice
//               may start as soon as this is done).  In the discrete form
//               the DR bits are these maps already: only the row fills, and
//               the clearing of the other parity's bits for the next slice
//   finalize -> (discrete form: drain of the slice's source set) sort +
//               unique of the slice's sampled sources, candidate check
//   merge    -> CSIP_t = NCSIP_{t-1} u N_t, ascending
//   estimate -> Eq8, then per candidate |ULE|^k, |URE|^k, Eq9, Algorithm 3's
//               test; the report goes straight into pinned host memory
//   slide    -> NCSIP_t compacted, SI counters updated, state advanced
// Every kernel reads its counts from device memory, so nothing waits for the
// host in between, and the two phases can be replayed as HIP graphs (one
// pair per slice parity).  srla_wait_report waits for the pipeline's end.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <atomic>
#include <vector>

#include "../../include/srla.h"
#include "srla_discrete.h"
#include "srla_noalloc.h"
#include "srla_scan_dedup.h"
#include "srla_scan_filter.h"
#include "srla_scan_part.h"
#include "srla_internal.h"

using namespace srla;

namespace {

// Hash parameters: SplitMix64 (Steele, Lea and Flood 2014) started at the
// hash seed; function f takes outputs 2f and 2f+1 as (a, b), in the order
// RH_0..RH_{u-1}, H1, H2, H3, H4.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

// smallest tau >= 0 with g * 2^tau >= theta: Eq1's ceil(log2(theta / g))
uint32_t eq1_tau(uint32_t theta, uint32_t g) {
  uint32_t tau = 0;
  while (((uint64_t)g << tau) < (uint64_t)theta) ++tau;
  return tau;
}

// ceil(rho * g) with rho = 0.99 (1 - e^(-1/3)) (Section 3.2)
uint32_t detect_threshold(uint32_t g) {
  const double rho = 0.99 * (1.0 - std::exp(-1.0 / 3.0));
  return (uint32_t)std::ceil(rho * (double)g);
}

bool config_ok(const srla_config_t* c) {
  if (!c) return false;
  const srla_geometry_t& g = c->geom;
  if (g.u < 1 || g.u > (uint32_t)kMaxU) return false;
  if (g.g < 1 || g.g > 64) return false;
  if (g.g_le < 64 || g.g_le % 64 != 0) return false;
  if (g.v_re < 1 || g.v_le < 1) return false;
  if (c->window_slices < 1 || c->window_slices > 32767) return false;
  if (c->threshold < 1) return false;
  if (c->max_candidates < 1 || c->max_candidates > 0xFFFFFFF0ull) return false;
  if ((c->flags & ~(uint32_t)(SRLA_CFG_TIMING | SRLA_CFG_SCAN_XCD | SRLA_CFG_GRAPH |
                              SRLA_CFG_DISCRETE | SRLA_CFG_LEAN_REPORT |
                              SRLA_CFG_SCAN_DEDUP | SRLA_CFG_SCAN_LDS_FILTER |
                              SRLA_CFG_OVERLAP_REPORT | SRLA_CFG_SCAN_PARTITION |
                              SRLA_CFG_HOLD_SCANS)) != 0)
    return false;
  if ((c->flags & SRLA_CFG_DISCRETE) && c->window_slices != 1) return false;
  const uint64_t le = (uint64_t)g.u * g.v_le * g.g_le;
  const uint64_t re = (uint64_t)g.u * g.v_re * g.g;
  if (le / g.u / g.g_le != g.v_le || re / g.u / g.g != g.v_re) return false;
  if (le > (1ull << 40) || re > (1ull << 40)) return false;
  // the partitioned form reads scan_blocks as its marking unit
  if ((c->flags & SRLA_CFG_SCAN_PARTITION) && !(c->flags & SRLA_CFG_DISCRETE) &&
      c->scan_blocks != 0 && !part_unit_ok(c->scan_blocks))
    return false;
  return true;
}

// DR indices per marking unit of a partitioned-scan monitor
uint32_t part_unit_of(const srla_config_t* c) {
  return (c->flags & SRLA_CFG_SCAN_PARTITION) && c->scan_blocks ? c->scan_blocks : kPartUnit;
}

enum Stage { ST_SCAN, ST_SWEEP, ST_FINALIZE, ST_ESTIMATE, ST_SLIDE, ST_REPORT, ST_N };

// the end-of-slice pipeline's two phases
// PH_FINISH_GO: the second phase when the next slice's first scan is enqueued
// behind a scan-start mark (the report copy then waits for that mark)
// PH_SORT: without the overlapped report, the sort of the closed slice's
// sampled sources: with held scans on the scan stream after the slice's
// scans, else on the pipeline stream as soon as they have appended every
// sampled source (beside the rest of the scan and the snapshot), ahead of
// the rest of the second phase
// PH_SLIDE: without the overlapped report, the tail of the second phase that
// the report does not wait for: Algorithm 3's carried list and SI counters,
// and the state moved to the next slice
// PH_SORT_SNAPSHOT: with held scans and no stage timing, PH_SORT and
// PH_SNAPSHOT in one launch (a launch boundary costs the stream ~20 us)
enum Phase { PH_SNAPSHOT = 0, PH_FINISH = 1, PH_FINISH_GO = 2, PH_SORT = 3, PH_SLIDE = 4,
             PH_SORT_SNAPSHOT = 5, PH_N = 6 };

struct TimedSpan {
  int stage;
  hipEvent_t a, b;
};

constexpr uint64_t kStageChunk = 1ull << 22;  // pairs per host-ingest chunk
// host report sets (slice mod kSets) and the cycle of (parity, set) pairs
constexpr int kSets = 3;
constexpr int kCycle = 6;

}  // namespace

struct srla_monitor {
  srla_config_t cfg{};
  Geo geo{};
  hipStream_t stream = nullptr;  // scans
  hipStream_t pipe = nullptr;    // end-of-slice pipeline (library-owned)
  hipStream_t pipe_use = nullptr;  // where the pipeline runs: pipe, or the
                                   // stream a group's members share
  int device = -1;               // the HIP device the monitor was created on
  bool pipe_own = false, copy_own = false;   // on a hardware queue of their own
  bool own_stream = false;
  uint64_t slice = 0;            // open slice
  bool poisoned = false;
  std::string err;

  // SEA and its per-slice views
  uint16_t* le = nullptr;        // stamps (not allocated in the discrete form)
  uint16_t* part_entries = nullptr;   // partitioned scan: sorted LE DR indices
  uint16_t* part_offs = nullptr;      //   their region offsets
  uint32_t* part_marks = nullptr;     //   and the marking bitmaps
  uint16_t* re = nullptr;
  bool discrete = false;         // k = 1 with one bit per DR
  uint64_t* lebits[2] = {nullptr, nullptr};  // discrete form: LE / SRE bits by slice parity
  uint64_t* rebits[2] = {nullptr, nullptr};
  uint64_t* sset[2] = {nullptr, nullptr};    // discrete form: sampled-source sets by parity
  uint32_t set_slots = 0;
  uint32_t* si_cnt = nullptr;    // [u][v_re][16] counters; SI bit = counter > 0
  uint64_t n_le = 0, n_re = 0, n_si = 0;
  // the snapshot of a closed slice, by slice parity: the next slice's
  // snapshot may run while this one's candidate work still reads it
  uint64_t* bitmap[2] = {nullptr, nullptr};   // LE DRs inside the window
  uint64_t* act[2] = {nullptr, nullptr};      // SRE DRs inside the window / after the slide
  unsigned long long* row_fill[2] = {nullptr, nullptr};
  unsigned long long* fill_part[2] = {nullptr, nullptr};   // the LE sweep's partial sums
  double* up[2] = {nullptr, nullptr};
  Counters* cnt = nullptr;
  PipeState* ps = nullptr;
  uint32_t* tcount = nullptr;    // [2] sampled-source counts by slice parity
  uint32_t* claim = nullptr;     // [2] tile-claim counters of the flat scan
  uint32_t* started = nullptr;   // scan-start mark: 1 + parity of the slice whose first scan
                                 // is about to start (overlapped report)
  uint32_t claim_slot = 0;       // the one the next flat scan uses

  // sources sampled, by slice parity, and the shared sort/finalize scratch
  uint32_t* touched[2] = {nullptr, nullptr};
  uint32_t* touched_tmp = nullptr;
  uint8_t* mark = nullptr;
  uint32_t* news = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* blockw = nullptr;
  uint64_t touched_cap = 0;
  uint64_t slice_pairs[2] = {0, 0};

  // candidate lists: slice parity p appends its new candidates to the carried
  // list carried[p] (CSIP) and leaves its own carried list in carried[p^1];
  // csip is scratch of that step
  uint32_t* csip = nullptr;
  uint32_t* carried[2] = {nullptr, nullptr};
  uint8_t* cflags = nullptr;
  uint32_t* cblockw = nullptr;
  uint64_t cap = 0;

  // pinned host side, one set per slice mod kSets (the report arrays and the
  // status blocks are written by kernels through their device-visible
  // addresses): a slice can be closed before the previous slice's report is
  // collected, and a slice's carried list goes into the next slice's set while
  // the host may still read the previous one
  HostStatus* h_status[kSets] = {};
  HostStatus* d_status[kSets] = {};
  uint64_t* h_row_fill64[kSets] = {};
  uint32_t* h_ip[kSets] = {};
  double* h_est[kSets] = {};
  uint8_t* h_flags[kSets] = {};
  // device copies of what h_est / h_flags hold (not with the overlapped
  // report): the estimate writes only the pieces that change
  double* d_mir_est[kSets] = {};
  uint8_t* d_mir_flags[kSets] = {};
  uint32_t* h_U[kSets] = {};
  uint8_t* h_W[kSets] = {};
  ReportPtrs d_report[kSets] = {};
  bool overlap_report = false;   // candidate work before the next slice's scans,
  ReportPtrs d_staging[2] = {};  // report staged here (by slice parity) and copied while
  uint32_t* report_n = nullptr;  // they run; [2] entries in each staged report

  // ordering: the snapshot phase runs on the scan stream, in order with the
  // scans; the second phase runs on the pipeline stream
  hipEvent_t ev_snap = nullptr;                 // after the last closed slice's snapshot phase
  hipEvent_t ev_scanned = nullptr;              // after the last closed slice's scans
  // after the partitioned scan's sampled-source appends (before its marking
  // and stamping); sampled_pending: the open slice's last scan recorded it
  hipEvent_t ev_sampled = nullptr;
  bool sampled_pending = false;
  hipEvent_t ev_sort = nullptr;                 // what the closed slice's sort waits for
  hipEvent_t ev_done[2] = {nullptr, nullptr};   // after the whole pipeline, by slice parity
  hipEvent_t ev_pub[2] = {nullptr, nullptr};    // the report and status are in host memory
  uint32_t n_pending = 0;         // closed slices whose reports are not collected (<= 2)
  int clock_khz = 0;              // rate of the device wall clock
  bool finish_deferred = false;   // the last closed slice's second phase is not enqueued yet

  // replayable pipeline: [phase][slice mod kCycle]
  bool use_graph = false;
  hipGraphExec_t graph[PH_N][kCycle] = {};

  // host-input ring: H2D copies on their own stream into two device chunks
  // (through two pinned bounce chunks when the caller's memory is pageable),
  // scans of the chunks on the scan stream
  hipStream_t copy = nullptr;
  uint32_t* h_stage[2] = {nullptr, nullptr};
  uint32_t* d_stage[2] = {nullptr, nullptr};
  hipEvent_t stage_ev[2] = {nullptr, nullptr};    // chunk copied to the device
  hipEvent_t scanned_ev[2] = {nullptr, nullptr};  // chunk scanned (device chunk free)
  bool stage_busy[2] = {false, false};
  bool scanned_set[2] = {false, false};
  int stage_next = 0;

  // timing (switched per call by srla_set_timing); timed[p]: the slice of
  // parity p was closed with timing on; time_scans: only the scans are timed
  bool timing = false;
  bool time_scans = false;
  bool timed[2] = {false, false};
  bool xcd_scan = false;
  bool dedup_scan = false;
  bool filter_scan = false;
  bool part_scan = false;
  bool hold_scans = false;       // scans wait for the closed slice's report
  std::vector<TimedSpan> spans;
  std::vector<hipEvent_t> ev_pool;
  double acc_ms[ST_N] = {0, 0, 0, 0, 0, 0};
  uint64_t scan_launches = 0, scan_pairs = 0, estimates = 0;
};

namespace {

int fail(srla_monitor* m, int code, const std::string& what) {
  if (m) m->err = what;
  return code;
}

int hip_fail(srla_monitor* m, hipError_t e, const char* where) {
  std::string s = std::string(where) + ": " + hipGetErrorString(e);
  if (m) m->poisoned = true;
  return fail(m, SRLA_E_DEVICE, s);
}

#define HIP_TRY(m, expr)                                   \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail((m), e_, #expr); \
  } while (0)

template <class T>
hipError_t dalloc(T** p, uint64_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

template <class T>
hipError_t halloc(T** p, uint64_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipHostMalloc((void**)p, count * sizeof(T), hipHostMallocDefault);
}

template <class T>
hipError_t dev_view(T* host, T** dev) {
  return hipHostGetDevicePointer((void**)dev, (void*)host, 0);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}
void hfree(void* p) {
  if (p) (void)hipHostFree(p);
}

uint64_t candidate_bytes(uint64_t cap) {
  // csip, two carried lists (u32), cflags (u8), block words
  return cap * (4 + 4 + 4 + 1) + 4 * compact_block_words(cap);
}

// device staging of the report when its copy overlaps the next slice's scans
// (two sets, by slice parity)
uint64_t staging_bytes(const srla_config_t* cfg) {
  if (!(cfg->flags & SRLA_CFG_OVERLAP_REPORT)) return 0;
  return 2 * cfg->max_candidates * ((cfg->flags & SRLA_CFG_LEAN_REPORT) ? 13 : 18) + 8;
}

// Makes stream st wait for ev, unless the host already sees ev complete (a
// wait costs the command processor a barrier packet even then).
hipError_t wait_unless_done(hipStream_t st, hipEvent_t ev) {
  const hipError_t q = hipEventQuery(ev);
  if (q == hipSuccess) return hipSuccess;
  (void)hipGetLastError();   // a not-ready query leaves no error behind
  return hipStreamWaitEvent(st, ev, 0);
}

uint64_t bitmap_words(uint64_t cells) { return (cells + 63) / 64 + 1; }

// device copies of the host report sets' est and flags arrays (9 bytes per
// candidate and set), except with the overlapped report
uint64_t mirror_bytes(const srla_config_t* cfg) {
  return (cfg->flags & SRLA_CFG_OVERLAP_REPORT) ? 0 : (uint64_t)kSets * cfg->max_candidates * 9;
}

// slots of the discrete form's sampled-source set: the power of two at least
// twice max_candidates (a slice's distinct sampled sources are its new
// candidates), within [2^12, 2^24]
uint32_t source_set_slots(uint64_t max_candidates) {
  uint64_t s = 1u << 12;
  while (s < 2 * max_candidates && s < (1u << 24)) s <<= 1;
  return (uint32_t)s;
}

// A stream with a hardware queue of its own.  HIP spreads ordinary streams
// over a small pool of hardware queues, so two streams of one process may land
// on the same queue and then run one after the other; a stream created with
// a CU mask is given its own queue.  The mask enables every CU (more bits than
// the device has CUs; the extra ones are ignored).  At most kOwnQueues such
// streams live in a process at once: many more hardware queues than the
// scheduler maps at a time make it switch between them (a serving mix of 64
// monitors ran 2.4 times slower with a queue each).  Beyond that, and if the
// masked stream cannot be created, an ordinary stream.  *own tells which.
constexpr int kOwnQueues = 8;
std::atomic<int> g_own_queues{0};

hipError_t create_queue_stream(hipStream_t* st, bool* own) {
  *own = false;
  if (g_own_queues.fetch_add(1) < kOwnQueues) {
    const std::vector<uint32_t> all(32, 0xFFFFFFFFu);
    if (hipExtStreamCreateWithCUMask(st, (uint32_t)all.size(), all.data()) == hipSuccess) {
      *own = true;
      return hipSuccess;
    }
    (void)hipGetLastError();
  }
  g_own_queues.fetch_sub(1);
  return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
}

void destroy_queue_stream(hipStream_t st, bool own) {
  (void)hipStreamDestroy(st);
  if (own) g_own_queues.fetch_sub(1);
}

hipEvent_t pooled_event(srla_monitor* m) {
  if (!m->ev_pool.empty()) {
    hipEvent_t e = m->ev_pool.back();
    m->ev_pool.pop_back();
    return e;
  }
  // a stage's timing events: only their timestamps are read, so their records
  // skip the system-scope release (a write-back of the caches that the next
  // kernel on the stream would wait for)
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) == hipSuccess) return e;
  (void)hipGetLastError();
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void span_begin(srla_monitor* m, hipStream_t st, hipEvent_t* a, bool scan = false) {
  *a = nullptr;
  if (!m->timing && !(scan && m->time_scans)) return;
  *a = pooled_event(m);
  if (*a) (void)hipEventRecord(*a, st);
}

// a: what span_begin returned (null: the span is not timed)
void span_end(srla_monitor* m, hipStream_t st, int stage, hipEvent_t a) {
  if (!a) return;
  hipEvent_t b = pooled_event(m);
  if (!b) { m->ev_pool.push_back(a); return; }
  (void)hipEventRecord(b, st);
  m->spans.push_back({stage, a, b});
}

// Adds the recorded spans to the stage totals: all of them (wait), or only
// those already complete, so that collecting one slice's report never waits
// for a later slice's work.
void collect_spans(srla_monitor* m, bool wait) {
  size_t kept = 0;
  for (auto& s : m->spans) {
    if (!wait && hipEventQuery(s.b) == hipErrorNotReady) {
      m->spans[kept++] = s;
      continue;
    }
    float ms = 0.f;
    if (hipEventSynchronize(s.b) == hipSuccess && hipEventElapsedTime(&ms, s.a, s.b) == hipSuccess)
      m->acc_ms[s.stage] += ms;
    m->ev_pool.push_back(s.a);
    m->ev_pool.push_back(s.b);
  }
  m->spans.resize(kept);
  (void)hipGetLastError();   // a not-ready query leaves no error behind
}

void drop_graphs(srla_monitor* m) {
  for (auto& ph : m->graph)
    for (auto& g : ph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Grows the sampled-source buffers (both parities) to hold `need` entries.
int reserve_touched(srla_monitor* m, uint64_t need) {
  if (need <= m->touched_cap) return SRLA_OK;
  if (need > 0xFFFFFFF0ull) return fail(m, SRLA_E_NOMEM, "slice holds more than 2^32 pairs");
  uint64_t cap = std::max<uint64_t>(need, m->touched_cap ? 2 * m->touched_cap : (1u << 20));
  cap = std::min<uint64_t>(cap, 0xFFFFFFF0ull);
  uint32_t *t0 = nullptr, *t1 = nullptr, *tt = nullptr, *nw = nullptr, *h = nullptr,
           *bw = nullptr;
  uint8_t* mk = nullptr;
  if (dalloc(&t0, cap) != hipSuccess || dalloc(&t1, cap) != hipSuccess ||
      dalloc(&tt, cap) != hipSuccess || dalloc(&nw, cap) != hipSuccess ||
      dalloc(&mk, cap) != hipSuccess || dalloc(&h, sort_aux_words()) != hipSuccess ||
      dalloc(&bw, compact_block_words(cap)) != hipSuccess) {
    dfree(t0); dfree(t1); dfree(tt); dfree(nw); dfree(mk); dfree(h); dfree(bw);
    (void)hipGetLastError();
    return fail(m, SRLA_E_NOMEM, "cannot grow the sampled-source buffers");
  }
  // both streams idle: the pending pipeline may still read the other parity
  HIP_TRY(m, hipStreamSynchronize(m->stream));
  HIP_TRY(m, hipStreamSynchronize(m->pipe_use));
  HIP_TRY(m, hipMemset(h, 0, sort_aux_words() * sizeof(uint32_t)));   // the sort's counters
  uint32_t* fresh[2] = {t0, t1};
  for (int p = 0; p < 2; ++p) {
    if (m->touched[p] && m->slice_pairs[p])
      HIP_TRY(m, hipMemcpy(fresh[p], m->touched[p], m->slice_pairs[p] * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice));
    dfree(m->touched[p]);
    m->touched[p] = fresh[p];
  }
  dfree(m->touched_tmp); dfree(m->news); dfree(m->mark); dfree(m->hist); dfree(m->blockw);
  m->touched_tmp = tt; m->news = nw; m->mark = mk; m->hist = h; m->blockw = bw;
  m->touched_cap = cap;
  drop_graphs(m);   // they hold the old buffers
  return SRLA_OK;
}

// Enqueues one phase of the end-of-slice pipeline of parity p on stream st.
// Every argument is fixed per (phase, parity), so the sequence can also be
// recorded once into a graph.
// The snapshot: the partial sums of |LDR(i)|^k and the activity maps of the
// closing slice (the discrete form: the row fills and Eq8 as well).
hipError_t enqueue_snapshot(srla_monitor* m, int p, hipStream_t st) {
  const Geo& geo = m->geo;
  hipError_t e = hipSuccess;
  hipEvent_t ta = nullptr;
  const bool spans = !m->use_graph;
  if (spans) span_begin(m, st, &ta);
  if (m->discrete) {
    e = launch_begin_close(m->ps, m->row_fill[p], geo.u, (uint32_t)p, st);
    if (e != hipSuccess) return e;
    // the closing slice's bits are its activity maps already; the other
    // parity's (the previous slice's) are cleared for the next slice's scans
    if (e == hipSuccess) e = launch_row_popcount(m->lebits[p], m->row_fill[p], geo, st);
    if (e == hipSuccess) e = launch_union_prob(m->row_fill[p], geo, m->up[p], st);
    if (e == hipSuccess)
      e = launch_fill_u32((uint32_t*)m->lebits[p ^ 1], 0u, 2 * bitmap_words(m->n_le), st);
    if (e == hipSuccess)
      e = launch_fill_u32((uint32_t*)m->rebits[p ^ 1], 0u, 4 * bitmap_words(m->n_re), st);
  } else {
    // one launch: the close, the sweeps; the row fills and Eq8 are folded
    // from the partial sums by the candidate check's first kernel
    e = launch_sweep(m->le, m->bitmap[p], m->fill_part[p], m->re, m->n_re, m->act[p], geo, m->ps,
                     (uint32_t)p, st);
  }
  if (spans) span_end(m, st, ST_SWEEP, ta);
  return e;
}

// The sort of the closing slice's sampled sources (drained from the source
// set first in the discrete form); it needs the slice's scans only.
hipError_t enqueue_sort(srla_monitor* m, int p, hipStream_t st) {
  hipError_t e = hipSuccess;
  uint32_t* tc = m->tcount + p;
  hipEvent_t ta = nullptr;
  const bool spans = !m->use_graph;
  if (spans) span_begin(m, st, &ta);
  if (m->discrete) e = launch_drain_set(m->sset[p], m->set_slots, m->touched[p], tc, st);
  if (e == hipSuccess)
    e = sort_u32(m->touched[p], m->touched_tmp, tc, m->hist, st);
  if (spans) span_end(m, st, ST_FINALIZE, ta);
  return e;
}

// Algorithm 3 after the estimate of the slice of parity p: the carried list
// NCSIP (the candidates whose SRE is still inside the window after the
// slide, as k_estimate flagged them), ascending, into carried[p ^ 1], and the
// SI counters.  next_ip: the next slice's report ip array, which then gets
// the carried list (the head of that report) at once.
hipError_t enqueue_slide(srla_monitor* m, int p, hipStream_t st, uint32_t* next_ip) {
  hipError_t e = hipSuccess;
  hipEvent_t ta = nullptr;
  const bool spans = !m->use_graph;
  uint32_t* cand = m->carried[p];
  if (spans) span_begin(m, st, &ta);
  e = compact_u32(m->cflags, 8u, cand, &m->cnt->n_cand, m->cap, m->csip, &m->cnt->n_keep,
                  m->cblockw, st);
  if (e == hipSuccess) e = launch_count_keep(m->cflags, m->ps, m->cnt, st);
  if (e == hipSuccess)
    e = launch_merge_runs(m->csip, &m->cnt->n_keep_a, &m->cnt->n_keep, m->carried[p ^ 1], st);
  if (e == hipSuccess) e = launch_si_update(cand, m->cflags, m->cnt, m->si_cnt, m->geo, st);
  if (e == hipSuccess && next_ip)
    e = launch_ip_precopy(m->carried[p ^ 1], &m->cnt->n_keep, next_ip, st);
  if (spans) span_end(m, st, ST_SLIDE, ta);
  return e;
}

// The candidate check of the closing slice's (sorted) sampled sources, and
// CSIP: the new candidates appended to the carried list.
hipError_t enqueue_check(srla_monitor* m, int p, hipStream_t st) {
  const Geo& geo = m->geo;
  hipError_t e = hipSuccess;
  uint32_t* tc = m->tcount + p;
  const uint64_t* re_act = m->discrete ? m->rebits[p] : m->act[p];
  hipEvent_t ta = nullptr;
  const bool spans = !m->use_graph;
  if (spans) span_begin(m, st, &ta);
  e = launch_finalize(m->touched[p], tc, re_act, m->si_cnt, geo, m->mark, m->cnt,
                      m->discrete ? nullptr : m->fill_part[p], m->row_fill[p], m->up[p], st);
  if (e == hipSuccess)
    e = compact_u32(m->mark, 1u, m->touched[p], tc, m->touched_cap, m->news, &m->cnt->n_new,
                    m->blockw, st);
  if (e == hipSuccess) e = launch_join(m->ps, m->news, m->cnt, m->cap, m->carried[p], st);
  if (spans) span_end(m, st, ST_FINALIZE, ta);
  return e;
}

// Eq9 for every candidate of CSIP, report entries to `out` (whose ip array
// holds the carried list already when skip_carried_ip).
hipError_t enqueue_estimate(srla_monitor* m, int p, const ReportPtrs& out, hipStream_t st,
                            bool skip_carried_ip) {
  const uint64_t* le_act = m->discrete ? m->lebits[p] : m->bitmap[p];
  const uint64_t* re_act = m->discrete ? m->rebits[p] : m->act[p];
  hipEvent_t ta = nullptr;
  const bool spans = !m->use_graph;
  if (spans) span_begin(m, st, &ta);
  const hipError_t e = launch_estimate(m->carried[p], m->cnt, m->ps, skip_carried_ip, le_act,
                                       re_act, m->up[p], m->row_fill[p], m->geo, m->cflags, out,
                                       st);
  if (spans) span_end(m, st, ST_ESTIMATE, ta);
  return e;
}

// The whole candidate work of the closing slice (the overlapped-report form
// runs it in one phase, into device staging): sort, check, Eq9 into `out`,
// then Algorithm 3's carried list and SI counters.
hipError_t enqueue_candidates(srla_monitor* m, int p, const ReportPtrs& out, hipStream_t st) {
  hipError_t e = enqueue_sort(m, p, st);
  if (e == hipSuccess) e = enqueue_check(m, p, st);
  if (e == hipSuccess) e = enqueue_estimate(m, p, out, st, false);
  if (e == hipSuccess) e = enqueue_slide(m, p, st, nullptr);
  return e;
}

// The two phases of the end-of-slice pipeline of parity p.  The first runs
// on the scan stream, right after the closing slice's scans, and the next
// slice's scans follow it there.  Normally it is the snapshot, and the
// candidate work, the report (written by the estimate kernel straight into
// host memory) and the status follow on the pipeline stream, beside those
// scans, and after them (PH_SLIDE) Algorithm 3's carried list and SI, which
// the report does not wait for; with held scans the sort, the candidate work
// and the report run on the scan stream as well (the next scans wait for
// them anyway), and only PH_SLIDE on the pipeline stream.  With
// SRLA_CFG_OVERLAP_REPORT the first
// phase also does the candidate work, into the parity's device staging
// arrays, and the status, and only the PCIe copy of the report overlaps the
// scans.  c: the slice's index mod kCycle, which fixes its parity (device
// arrays) and its report set (host arrays).
hipError_t enqueue_phase(srla_monitor* m, int phase, int c, hipStream_t st) {
  hipError_t e = hipSuccess;
  hipEvent_t ta = nullptr;
  const bool spans = !m->use_graph;
  const int p = c & 1, q = c % kSets, q_next = (c + 1) % kSets;
  if (phase == PH_SORT) return enqueue_sort(m, p, st);
  if (phase == PH_SORT_SNAPSHOT) {
    e = enqueue_sort(m, p, st);
    return e == hipSuccess ? enqueue_snapshot(m, p, st) : e;
  }
  if (phase == PH_SLIDE) {
    e = enqueue_slide(m, p, st, m->d_report[q_next].ip);
    if (e == hipSuccess) e = launch_advance(m->cnt, m->tcount + p, m->ps, st);
    return e;
  }
  if (phase == PH_SNAPSHOT) {
    e = enqueue_snapshot(m, p, st);
    if (e == hipSuccess && m->overlap_report) {
      e = enqueue_candidates(m, p, m->d_staging[p], st);
      if (spans) span_begin(m, st, &ta);
      if (e == hipSuccess)
        e = launch_status(m->cnt, m->tcount + p, m->up[p], m->row_fill[p], m->geo.u, m->ps,
                          (uint32_t)p,
                          m->d_status[q], m->report_n + p, st);
      if (spans) span_end(m, st, ST_SLIDE, ta);
    }
    return e;
  }
  if (!m->overlap_report) {
    e = enqueue_check(m, p, st);
    if (e == hipSuccess) e = enqueue_estimate(m, p, m->d_report[q], st, true);
  }
  if (spans) span_begin(m, st, &ta);
  if (m->overlap_report) {
    // PH_FINISH_GO: the next slice (parity p ^ 1) has its first scan behind a mark
    const uint32_t expect = phase == PH_FINISH_GO ? (uint32_t)(p ^ 1) + 1u : 0u;
    if (e == hipSuccess)
      e = launch_report_copy(m->report_n + p, m->d_staging[p], m->d_report[q], m->started, expect,
                             st);
    if (e == hipSuccess) e = launch_mark_done(m->d_status[q], st);
  } else if (e == hipSuccess) {
    e = launch_publish(m->cnt, m->tcount + p, m->up[p], m->row_fill[p], m->geo.u, m->ps,
                       (uint32_t)p, m->d_status[q], st);
  }
  if (spans) span_end(m, st, ST_REPORT, ta);
  return e;
}

// Runs one phase of the slice with index mod kCycle c on stream st: directly,
// or through its graph (recorded on first use, on the pipeline stream, and
// launched on st).
int run_phase(srla_monitor* m, int phase, int c, hipStream_t st) {
  if (!m->use_graph) {
    HIP_TRY(m, enqueue_phase(m, phase, c, st));
    return SRLA_OK;
  }
  hipGraphExec_t& exec = m->graph[phase][c];
  if (!exec) {
    hipGraph_t g = nullptr;
    HIP_TRY(m, hipStreamBeginCapture(m->pipe, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_phase(m, phase, c, m->pipe);
    const hipError_t ec = hipStreamEndCapture(m->pipe, &g);
    HIP_TRY(m, e);
    HIP_TRY(m, ec);
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(m, ei);
  }
  HIP_TRY(m, hipGraphLaunch(exec, st));
  return SRLA_OK;
}

void release(srla_monitor* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  if (m->pipe_use && m->pipe_use != m->pipe) (void)hipStreamSynchronize(m->pipe_use);
  if (m->pipe) (void)hipStreamSynchronize(m->pipe);
  collect_spans(m, true);
  drop_graphs(m);
  dfree(m->le); dfree(m->re); dfree(m->si_cnt);
  dfree(m->part_entries); dfree(m->part_offs); dfree(m->part_marks);
  for (int i = 0; i < 2; ++i) { dfree(m->lebits[i]); dfree(m->rebits[i]); dfree(m->sset[i]); } 
  for (int i = 0; i < 2; ++i) { dfree(m->bitmap[i]); dfree(m->act[i]); }
  for (int i = 0; i < 2; ++i) { dfree(m->row_fill[i]); dfree(m->fill_part[i]); dfree(m->up[i]); }
  dfree(m->cnt); dfree(m->ps);
  dfree(m->tcount);
  dfree(m->claim);
  dfree(m->started);
  dfree(m->touched[0]); dfree(m->touched[1]); dfree(m->touched_tmp); dfree(m->mark);
  dfree(m->news); dfree(m->hist); dfree(m->blockw);
  dfree(m->csip); dfree(m->carried[0]); dfree(m->carried[1]); dfree(m->cflags);
  dfree(m->cblockw);
  for (auto& sg : m->d_staging) {
    dfree(sg.ip); dfree(sg.est); dfree(sg.flags); dfree(sg.U); dfree(sg.W);
  }
  dfree(m->report_n);
  for (int q = 0; q < kSets; ++q) {
    hfree(m->h_status[q]); hfree(m->h_ip[q]); hfree(m->h_est[q]); hfree(m->h_flags[q]);
    dfree(m->d_mir_est[q]); dfree(m->d_mir_flags[q]);
    hfree(m->h_U[q]); hfree(m->h_W[q]);
    delete[] m->h_row_fill64[q];
  }
  for (int q = 0; q < 2; ++q) {
    if (m->ev_done[q]) (void)hipEventDestroy(m->ev_done[q]);
    if (m->ev_pub[q]) (void)hipEventDestroy(m->ev_pub[q]);
  }
  for (int i = 0; i < 2; ++i) {
    hfree(m->h_stage[i]);
    dfree(m->d_stage[i]);
    if (m->stage_ev[i]) (void)hipEventDestroy(m->stage_ev[i]);
    if (m->scanned_ev[i]) (void)hipEventDestroy(m->scanned_ev[i]);
  }
  for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
  if (m->ev_snap) (void)hipEventDestroy(m->ev_snap);
  if (m->ev_scanned) (void)hipEventDestroy(m->ev_scanned);
  if (m->ev_sampled) (void)hipEventDestroy(m->ev_sampled);
  if (m->pipe) destroy_queue_stream(m->pipe, m->pipe_own);
  if (m->copy) {
    (void)hipStreamSynchronize(m->copy);
    destroy_queue_stream(m->copy, m->copy_own);
  }
  if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

}  // namespace

extern "C" {

uint64_t srla_footprint_bytes(const srla_config_t* cfg) {
  if (!config_ok(cfg)) return 0;
  const srla_geometry_t& g = cfg->geom;
  const uint64_t le = (uint64_t)g.u * g.v_le * g.g_le;
  const uint64_t re = (uint64_t)g.u * g.v_re * g.g;
  const uint64_t si = (uint64_t)g.u * g.v_re;
  if (cfg->flags & SRLA_CFG_DISCRETE)
    return 16 * bitmap_words(le) + 32 * bitmap_words(re) +
           16 * (uint64_t)source_set_slots(cfg->max_candidates) + 64 * si + 16 * g.u + 16 +
           staging_bytes(cfg) + mirror_bytes(cfg) +
           sizeof(Counters) + sizeof(PipeState) + 8 + 8 + 8 + candidate_bytes(cfg->max_candidates);
  const uint64_t part = (cfg->flags & SRLA_CFG_SCAN_PARTITION)
                            ? 2 * (part_entry_words() + part_offset_words(le)) +
                                  4 * part_mark_words(le, kPartChunks, part_unit_of(cfg))
                            : 0;
  return part + staging_bytes(cfg) + mirror_bytes(cfg) + 2 * le + 16 * bitmap_words(le) +
         2 * (re + 8) +
         32 * bitmap_words(re) + 64 * si + 16 * g.u + 16 * kFillSlots * g.u + 16 + sizeof(Counters) + sizeof(PipeState) + 8 + 8 + 8 +
         candidate_bytes(cfg->max_candidates);
}

int srla_admit(const srla_config_t* cfgs, uint32_t n, uint64_t budget_bytes, uint8_t* admitted,
               uint64_t* used_bytes) {
  if ((n && (!cfgs || !admitted)) || !used_bytes) return SRLA_E_INVAL;
  for (uint32_t i = 0; i < n; ++i)
    if (!config_ok(&cfgs[i])) return SRLA_E_INVAL;
  uint64_t used = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint64_t fp = srla_footprint_bytes(&cfgs[i]);
    admitted[i] = (fp <= budget_bytes - used) ? 1 : 0;   // used <= budget always holds
    if (admitted[i]) used += fp;
  }
  *used_bytes = used;
  return SRLA_OK;
}

int srla_create(const srla_config_t* cfg, void* hip_stream, srla_monitor_t** out) {
  if (!out) return SRLA_E_INVAL;
  if (!config_ok(cfg)) return SRLA_E_INVAL;
  srla_monitor* m = new (std::nothrow) srla_monitor();
  if (!m) return SRLA_E_NOMEM;
  m->cfg = *cfg;
  m->timing = (cfg->flags & SRLA_CFG_TIMING) != 0;
  m->xcd_scan = (cfg->flags & SRLA_CFG_SCAN_XCD) != 0;
  m->use_graph = (cfg->flags & SRLA_CFG_GRAPH) != 0;
  m->discrete = (cfg->flags & SRLA_CFG_DISCRETE) != 0;
  m->dedup_scan = (cfg->flags & SRLA_CFG_SCAN_DEDUP) != 0;
  m->filter_scan = (cfg->flags & SRLA_CFG_SCAN_LDS_FILTER) != 0;
  m->part_scan = (cfg->flags & SRLA_CFG_SCAN_PARTITION) != 0 && !m->discrete;
  m->overlap_report = (cfg->flags & SRLA_CFG_OVERLAP_REPORT) != 0;
  m->hold_scans = (cfg->flags & SRLA_CFG_HOLD_SCANS) != 0 && !m->overlap_report;

  const srla_geometry_t& g = cfg->geom;
  Geo& geo = m->geo;
  geo.u = g.u; geo.v_re = g.v_re; geo.g = g.g; geo.v_le = g.v_le; geo.G = g.g_le;
  geo.k = cfg->window_slices;
  geo.theta = cfg->threshold;
  const uint32_t tau = eq1_tau(cfg->threshold, g.g);
  geo.tau_mask = tau >= 32 ? 0xFFFFFFFFu : ((1u << tau) - 1u);
  geo.t_re = detect_threshold(g.g);
  geo.words = g.g_le / 64;
  SplitMix64 sm{g.hash_seed};
  for (uint32_t f = 0; f < g.u + 4; ++f) {
    HashFn h;
    h.a = sm.next();
    h.b = sm.next();
    if (f < g.u) geo.rh[f] = h;
    else if (f == g.u) geo.h1 = h;
    else if (f == g.u + 1) geo.h2 = h;
    else if (f == g.u + 2) geo.h3 = h;
    else geo.h4 = h;
  }

  int rc = SRLA_OK;
  auto nomem = [&](hipError_t e) {
    if (e != hipSuccess) {
      (void)hipGetLastError();
      rc = SRLA_E_NOMEM;
    }
  };
  if (hip_stream) {
    m->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
      release(m);
      return SRLA_E_DEVICE;
    }
    m->own_stream = true;
  }
  // the pipeline stream runs beside the scan stream: a queue of its own
  if (create_queue_stream(&m->pipe, &m->pipe_own) != hipSuccess) {
    release(m);
    return SRLA_E_DEVICE;
  }
  m->pipe_use = m->pipe;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      release(m);
      return SRLA_E_DEVICE;
    }
    m->device = dev;
    if (hipDeviceGetAttribute(&m->clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
      m->clock_khz = 0;
    (void)hipGetLastError();
    // the allocation-free scan's scratch address on this device, looked up once
    if (noalloc_setup(dev) != hipSuccess) {
      (void)hipGetLastError();
      release(m);
      return SRLA_E_DEVICE;
    }
  }
  m->n_le = (uint64_t)g.u * g.v_le * g.g_le;
  m->n_re = (uint64_t)g.u * g.v_re * g.g;
  m->n_si = (uint64_t)g.u * g.v_re;
  m->cap = cfg->max_candidates;
  if (m->discrete) {
    m->set_slots = source_set_slots(cfg->max_candidates);
    for (int i = 0; i < 2 && !rc; ++i) {
      nomem(dalloc(&m->lebits[i], bitmap_words(m->n_le)));
      if (!rc) nomem(dalloc(&m->rebits[i], 2 * bitmap_words(m->n_re)));
      if (!rc) nomem(dalloc(&m->sset[i], m->set_slots));
    }
  } else {
    nomem(dalloc(&m->le, m->n_le));
    if (!rc) nomem(dalloc(&m->re, m->n_re + 8));
    for (int i = 0; i < 2 && !rc; ++i) {
      nomem(dalloc(&m->bitmap[i], bitmap_words(m->n_le)));
      if (!rc) nomem(dalloc(&m->act[i], 2 * bitmap_words(m->n_re)));
    }
    if (!rc && m->part_scan) nomem(dalloc(&m->part_entries, part_entry_words()));
    if (!rc && m->part_scan) nomem(dalloc(&m->part_offs, part_offset_words(m->n_le)));
    if (!rc && m->part_scan)
      nomem(dalloc(&m->part_marks, part_mark_words(m->n_le, kPartChunks, part_unit_of(&m->cfg))));
  }
  if (!rc) nomem(dalloc(&m->si_cnt, 16 * m->n_si));
  for (int i = 0; i < 2 && !rc; ++i) {
    nomem(dalloc(&m->row_fill[i], g.u));
    if (!rc && !m->discrete) nomem(dalloc(&m->fill_part[i], (uint64_t)g.u * kFillSlots));
    if (!rc) nomem(dalloc(&m->up[i], 1));
  }
  if (!rc) nomem(dalloc(&m->cnt, 1));
  if (!rc) nomem(dalloc(&m->ps, 1));
  if (!rc) nomem(dalloc(&m->tcount, 2));
  if (!rc) nomem(dalloc(&m->claim, 2));
  if (!rc) nomem(dalloc(&m->started, 1));
  if (!rc) nomem(dalloc(&m->csip, m->cap));
  if (!rc) nomem(dalloc(&m->carried[0], m->cap));
  if (!rc) nomem(dalloc(&m->carried[1], m->cap));
  if (!rc) nomem(dalloc(&m->cflags, m->cap));
  if (!rc) nomem(dalloc(&m->cblockw, compact_block_words(m->cap)));
  if (!rc && m->overlap_report) {
    nomem(dalloc(&m->report_n, 2));
    for (auto& sg : m->d_staging) {
      if (!rc) nomem(dalloc(&sg.ip, m->cap));
      if (!rc) nomem(dalloc(&sg.est, m->cap));
      if (!rc) nomem(dalloc(&sg.flags, m->cap));
      if (!rc && !(cfg->flags & SRLA_CFG_LEAN_REPORT)) nomem(dalloc(&sg.U, m->cap));
      if (!rc && !(cfg->flags & SRLA_CFG_LEAN_REPORT)) nomem(dalloc(&sg.W, m->cap));
    }
  }
  const bool weights = (cfg->flags & SRLA_CFG_LEAN_REPORT) == 0;
  for (int q = 0; q < kSets && !rc; ++q) {
    nomem(halloc(&m->h_status[q], 1));
    if (!rc) nomem(halloc(&m->h_ip[q], m->cap));
    if (!rc) nomem(halloc(&m->h_est[q], m->cap));
    if (!rc) nomem(halloc(&m->h_flags[q], m->cap));
    if (!rc && weights) nomem(halloc(&m->h_U[q], m->cap));
    if (!rc && weights) nomem(halloc(&m->h_W[q], m->cap));
    if (!rc) {
      m->h_row_fill64[q] = new (std::nothrow) uint64_t[g.u];
      if (!m->h_row_fill64[q]) rc = SRLA_E_NOMEM;
    }
    // the host arrays and their device copies start out equal (all zero)
    if (!rc) {
      std::memset(m->h_est[q], 0, m->cap * sizeof(double));
      std::memset(m->h_flags[q], 0, m->cap);
    }
    if (!rc && !m->overlap_report) {
      nomem(dalloc(&m->d_mir_est[q], m->cap));
      if (!rc) nomem(dalloc(&m->d_mir_flags[q], m->cap));
      if (!rc && (hipMemset(m->d_mir_est[q], 0, m->cap * sizeof(double)) != hipSuccess ||
                  hipMemset(m->d_mir_flags[q], 0, m->cap) != hipSuccess))
        rc = SRLA_E_DEVICE;
      m->d_report[q].mir_est = m->d_mir_est[q];
      m->d_report[q].mir_flags = m->d_mir_flags[q];
    }
    if (!rc && (dev_view(m->h_status[q], &m->d_status[q]) != hipSuccess ||
                dev_view(m->h_ip[q], &m->d_report[q].ip) != hipSuccess ||
                dev_view(m->h_est[q], &m->d_report[q].est) != hipSuccess ||
                dev_view(m->h_flags[q], &m->d_report[q].flags) != hipSuccess ||
                (weights && dev_view(m->h_U[q], &m->d_report[q].U) != hipSuccess) ||
                (weights && dev_view(m->h_W[q], &m->d_report[q].W) != hipSuccess)))
      rc = SRLA_E_DEVICE;
  }
  for (int q = 0; q < 2 && !rc; ++q) {
    if (!rc && hipEventCreateWithFlags(&m->ev_done[q], hipEventDisableTiming) != hipSuccess)
      rc = SRLA_E_DEVICE;
    if (!rc && hipEventCreateWithFlags(&m->ev_pub[q], hipEventDisableTiming) != hipSuccess)
      rc = SRLA_E_DEVICE;
  }
  if (!rc && hipEventCreateWithFlags(&m->ev_sampled, hipEventDisableTiming) != hipSuccess)
    rc = SRLA_E_DEVICE;
  if (!rc && hipEventCreateWithFlags(&m->ev_scanned, hipEventDisableTiming) != hipSuccess)
    rc = SRLA_E_DEVICE;
  if (!rc && hipEventCreateWithFlags(&m->ev_snap, hipEventDisableTiming) != hipSuccess)
    rc = SRLA_E_DEVICE;
  if (rc) {
    release(m);
    return rc;
  }
  // DRinit for every DR (stamp 0 = never set), SI = 0, counters = 0, slice 0
  hipError_t e = hipSuccess;
  if (m->discrete) {
    // every bit clear; the "after the slide" half of each SRE word pair stays
    // clear for good (at k = 1 no DR is inside the window after the slide)
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = launch_fill_u32((uint32_t*)m->lebits[i], 0u, 2 * bitmap_words(m->n_le), m->stream);
      if (e == hipSuccess)
        e = launch_fill_u32((uint32_t*)m->rebits[i], 0u, 4 * bitmap_words(m->n_re), m->stream);
      if (e == hipSuccess)
        e = launch_fill_u32((uint32_t*)m->sset[i], 0u, 2ull * m->set_slots, m->stream);
    }
  } else {
    if (e == hipSuccess) e = launch_fill_u32((uint32_t*)m->le, 0u, m->n_le / 2, m->stream);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t*)m->re, 0u, (m->n_re + 8) / 2, m->stream);
  }
  if (e == hipSuccess) e = launch_fill_u32(m->si_cnt, 0u, 16 * m->n_si, m->stream);
  for (int i = 0; i < 2 && e == hipSuccess && !m->discrete; ++i)
    e = launch_fill_u32((uint32_t*)m->fill_part[i], 0u, 2ull * m->geo.u * kFillSlots, m->stream);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)m->cnt, 0u, sizeof(Counters) / 4, m->stream);
  if (e == hipSuccess) e = launch_fill_u32(m->tcount, 0u, 2, m->stream);
  if (e == hipSuccess) e = launch_fill_u32(m->claim, 0u, 2, m->stream);
  if (e == hipSuccess) e = launch_fill_u32(m->started, 0u, 1, m->stream);
  if (e == hipSuccess) {
    PipeState ps0{};
    ps0.now = stamp_code(0);
    e = hipMemcpyAsync(m->ps, &ps0, sizeof(ps0), hipMemcpyHostToDevice, m->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    release(m);
    return SRLA_E_DEVICE;
  }
  if (reserve_touched(m, 1u << 16) != SRLA_OK) {
    release(m);
    return SRLA_E_NOMEM;
  }
  *out = m;
  return SRLA_OK;
}

}  // extern "C"

namespace {

// Algorithm 2 for n device-resident pairs of the open slice (parity p) in the
// monitor's scan form
// mark != 0: the scan-start mark to set as this scan starts (by the flat
// scan kernel itself, else by a marker kernel just before the scan)
hipError_t enqueue_scan(srla_monitor* m, const uint32_t* pairs, uint64_t n, int p,
                        uint32_t mark) {
  const uint16_t code = stamp_code(m->slice);
  if (mark != 0u && (m->discrete || m->part_scan || m->dedup_scan || m->filter_scan)) {
    const hipError_t e = launch_mark_scan(m->started, mark, m->stream);
    if (e != hipSuccess) return e;
  }
  if (m->discrete)
    return launch_scan_bits(pairs, n, m->geo, m->lebits[p], m->rebits[p], m->sset[p],
                            m->set_slots, m->touched[p], m->tcount + p, m->cfg.scan_blocks,
                            m->stream);
  m->sampled_pending = m->part_scan && !m->overlap_report && !m->hold_scans;
  if (m->part_scan)
    return launch_scan_partition(pairs, n, m->geo, code, m->le, m->re, m->touched[p],
                                 m->tcount + p, m->part_entries, m->part_offs, m->part_marks,
                                 m->stream, kPartChunks, m->ps, (uint32_t)p,
                                 part_unit_of(&m->cfg),
                                 m->sampled_pending ? m->ev_sampled : nullptr);
  if (m->dedup_scan)
    return launch_scan_dedup(pairs, n, m->geo, code, m->le, m->re, m->touched[p],
                             m->tcount + p, m->xcd_scan, m->cfg.scan_blocks, m->stream);
  if (m->filter_scan)
    return launch_scan_lds_filter(pairs, n, m->geo, code, m->le, m->re, m->touched[p],
                                  m->tcount + p, m->claim, &m->claim_slot, m->cfg.scan_blocks,
                                  m->stream);
  return launch_scan(pairs, n, m->geo, code, m->le, m->re, m->touched[p], m->tcount + p,
                     m->claim, &m->claim_slot, m->xcd_scan, m->cfg.scan_blocks, m->stream,
                     m->started, mark);
}

// Enqueues the second phase of the last closed slice's pipeline on the
// pipeline stream, after its first phase (ev_snap, recorded on the scan
// stream), and its completion event.  With the overlapped report this is
// done once the next slice's first scan is already enqueued on the scan
// stream, right behind ev_snap, so the report's PCIe copy starts after that
// scan has been dispatched: a kernel that streams writes into host memory
// delays the dispatch of kernels of other queues by hundreds of microseconds
// (the command processor reads queue packets and signals in host memory
// behind those writes), so the scan has to be under way before the copy.
int enqueue_finish(srla_monitor* m, bool go) {
  const int pc = (int)((m->slice - 1) & 1);   // parity of the closed slice
  const int cc = (int)((m->slice - 1) % kCycle);
  // timed as the slice was when it was closed
  struct TimingAs {
    srla_monitor* m;
    bool saved;
    TimingAs(srla_monitor* mm, bool t) : m(mm), saved(mm->timing) { m->timing = t; }
    ~TimingAs() { m->timing = saved; }
  } timing_as(m, m->timed[pc]);
  hipEvent_t ta;
  if (!m->overlap_report && !m->hold_scans) {
    // the sort needs the slice's scans only: it runs beside the snapshot
    HIP_TRY(m, hipStreamWaitEvent(m->pipe_use, m->ev_sort, 0));
    if (m->use_graph) span_begin(m, m->pipe_use, &ta);
    const int rs = run_phase(m, PH_SORT, cc, m->pipe_use);
    if (rs) return rs;
    if (m->use_graph) span_end(m, m->pipe_use, ST_FINALIZE, ta);
  }
  // with held scans the candidate work and the report run on the scan
  // stream, in order after the snapshot, and the next slice's scans follow
  // them there: no wait between streams on the way from the last scan to the
  // report and on to the next scan, and the end-of-slice work has the GPU to
  // itself (the scans overlap only Algorithm 3's carried list and SI update
  // on the pipeline stream)
  hipStream_t fs = m->hold_scans ? m->stream : m->pipe_use;
  if (!m->hold_scans) HIP_TRY(m, hipStreamWaitEvent(m->pipe_use, m->ev_snap, 0));
  if (m->use_graph) span_begin(m, fs, &ta);
  int rc = run_phase(m, go ? PH_FINISH_GO : PH_FINISH, cc, fs);
  if (rc) return rc;
  if (m->use_graph) span_end(m, fs, m->overlap_report ? ST_REPORT : ST_ESTIMATE, ta);
  HIP_TRY(m, hipEventRecord(m->ev_pub[pc], fs));
  if (!m->overlap_report) {
    if (m->hold_scans) HIP_TRY(m, hipStreamWaitEvent(m->pipe_use, m->ev_pub[pc], 0));
    if (m->use_graph) span_begin(m, m->pipe_use, &ta);
    rc = run_phase(m, PH_SLIDE, cc, m->pipe_use);
    if (rc) return rc;
    if (m->use_graph) span_end(m, m->pipe_use, ST_SLIDE, ta);
  }
  HIP_TRY(m, hipEventRecord(m->ev_done[pc], m->pipe_use));
  m->finish_deferred = false;
  return SRLA_OK;
}

// true if p is page-locked host memory that the DMA engines can read directly
bool host_pinned(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();   // pageable memory: not known to the runtime
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

}  // namespace

extern "C" {

int srla_scan(srla_monitor_t* m, const uint32_t* pairs, uint64_t n, int on_device) {
  if (!m) return SRLA_E_INVAL;
  if (m->poisoned) return fail(m, SRLA_E_STATE, "monitor is poisoned by an earlier error");
  if (n == 0) return SRLA_OK;
  if (!pairs) return fail(m, SRLA_E_INVAL, "pairs is NULL");
  const int p = (int)(m->slice & 1);
  int rc = reserve_touched(m, m->slice_pairs[p] + n);
  if (rc) return rc;
  // the first scan after an overlapped close sets the scan-start mark; the
  // deferred second phase of the closed slice is enqueued after it, and its
  // report copy waits for the mark (see enqueue_finish)
  bool go = m->finish_deferred;
  const uint32_t mark = go ? (uint32_t)p + 1u : 0u;
  if (on_device) {
    hipEvent_t a;
    span_begin(m, m->stream, &a, true);
    HIP_TRY(m, enqueue_scan(m, pairs, n, p, mark));
    span_end(m, m->stream, ST_SCAN, a);
    // the partitioned scan records its own end; other forms get a marker
    if (!m->part_scan || m->discrete)
      HIP_TRY(m, launch_scan_end(m->ps, (uint32_t)p, m->stream));
    m->slice_pairs[p] += n;
    if (m->timing || m->time_scans) {
      m->scan_launches++;
      m->scan_pairs += n;
    }
    return go ? enqueue_finish(m, true) : SRLA_OK;
  }
  // host input: chunk by chunk, H2D copies on the copy stream overlapping the
  // scans of earlier chunks on the scan stream
  if (!m->copy) {
    if (create_queue_stream(&m->copy, &m->copy_own) != hipSuccess) {
      (void)hipGetLastError();
      return fail(m, SRLA_E_DEVICE, "cannot create the host-ingest stream");
    }
  }
  for (int i = 0; i < 2; ++i) {
    if (!m->h_stage[i]) {
      if (halloc(&m->h_stage[i], 2 * kStageChunk) != hipSuccess ||
          dalloc(&m->d_stage[i], 2 * kStageChunk) != hipSuccess ||
          hipEventCreateWithFlags(&m->stage_ev[i], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&m->scanned_ev[i], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(m, SRLA_E_NOMEM, "cannot allocate the host-ingest ring");
      }
    }
  }
  const bool pinned = host_pinned(pairs);
  int last = -1;
  for (uint64_t off = 0; off < n; off += kStageChunk) {
    const uint64_t cnt = std::min(kStageChunk, n - off);
    const uint64_t bytes = cnt * 2 * sizeof(uint32_t);
    const int b = m->stage_next;
    m->stage_next ^= 1;
    // the device chunk is free once its previous scan has run
    if (m->scanned_set[b]) HIP_TRY(m, hipStreamWaitEvent(m->copy, m->scanned_ev[b], 0));
    const uint32_t* src = pairs + 2 * off;
    if (!pinned) {
      // the pinned bounce chunk is free once its previous copy has run
      if (m->stage_busy[b]) HIP_TRY(m, hipEventSynchronize(m->stage_ev[b]));
      std::memcpy(m->h_stage[b], src, bytes);
      src = m->h_stage[b];
    }
    HIP_TRY(m, hipMemcpyAsync(m->d_stage[b], src, bytes, hipMemcpyHostToDevice, m->copy));
    HIP_TRY(m, hipEventRecord(m->stage_ev[b], m->copy));
    m->stage_busy[b] = true;
    HIP_TRY(m, hipStreamWaitEvent(m->stream, m->stage_ev[b], 0));
    hipEvent_t a;
    span_begin(m, m->stream, &a, true);
    HIP_TRY(m, enqueue_scan(m, m->d_stage[b], cnt, p, go ? mark : 0u));
    span_end(m, m->stream, ST_SCAN, a);
    if (!m->part_scan || m->discrete)
      HIP_TRY(m, launch_scan_end(m->ps, (uint32_t)p, m->stream));
    if (go) {
      rc = enqueue_finish(m, true);
      if (rc) return rc;
      go = false;
    }
    HIP_TRY(m, hipEventRecord(m->scanned_ev[b], m->stream));
    m->scanned_set[b] = true;
    m->slice_pairs[p] += cnt;
    if (m->timing || m->time_scans) {
      m->scan_launches++;
      m->scan_pairs += cnt;
    }
    last = b;
  }
  // the caller may reuse its buffer once this returns: wait for the copies
  // that read it directly
  if (pinned && last >= 0) HIP_TRY(m, hipEventSynchronize(m->stage_ev[last]));
  return SRLA_OK;
}

int srla_scan_noalloc(srla_monitor_t* m, const uint32_t* pairs, uint64_t n) {
  if (!m) return SRLA_E_INVAL;
  if (m->poisoned) return fail(m, SRLA_E_STATE, "monitor is poisoned by an earlier error");
  if (n == 0) return SRLA_OK;
  if (!pairs) return fail(m, SRLA_E_INVAL, "pairs is NULL");
  if (m->discrete || m->overlap_report)
    return fail(m, SRLA_E_INVAL,
                "srla_scan_noalloc: not for discrete or overlapped-report monitors");
  const int p = (int)(m->slice & 1);
  if (m->slice_pairs[p] + n > m->touched_cap)
    return fail(m, SRLA_E_INVAL,
                "srla_scan_noalloc: the slice's pairs exceed the sampled-source capacity");
  uint8_t* base = static_cast<uint8_t*>(noalloc_scratch(m->device));
  if (!base) return fail(m, SRLA_E_DEVICE, "srla_scan_noalloc: no scratch on this device");
  uint16_t* entries = reinterpret_cast<uint16_t*>(base);
  uint32_t* marks = reinterpret_cast<uint32_t*>(base + kNoAllocEntryBytes);
  uint16_t* offs = reinterpret_cast<uint16_t*>(base + kNoAllocEntryBytes + kNoAllocMarkBytes);
  m->sampled_pending = !m->hold_scans;
  HIP_TRY(m, launch_scan_partition(pairs, n, m->geo, stamp_code(m->slice), m->le, m->re,
                                   m->touched[p], m->tcount + p, entries, offs, marks,
                                   m->stream, kNoAllocChunks, m->ps, (uint32_t)p, kPartUnit,
                                   m->sampled_pending ? m->ev_sampled : nullptr));
  m->slice_pairs[p] += n;
  return SRLA_OK;
}

int srla_close_slice(srla_monitor_t* m) {
  if (!m) return SRLA_E_INVAL;
  if (m->poisoned) return fail(m, SRLA_E_STATE, "monitor is poisoned by an earlier error");
  if (m->n_pending >= 2)
    return fail(m, SRLA_E_STATE, "the reports of two closed slices have not been collected");
  const int p = (int)(m->slice & 1);
  m->timed[p] = m->timing;
  // the previous slice's second phase is enqueued first; then the scan stream
  // waits for the work this slice's first phase would overwrite: with the
  // overlapped report, the report copy of the slice two back (it reads the
  // staging set this slice writes), normally long finished; in the discrete
  // form, the previous slice's second phase (the snapshot clears the bits it
  // reads).  Otherwise the snapshot writes its parity's arrays only, which
  // the slice two back has finished with (see below), and runs at once.
  if (m->finish_deferred) {
    const int rc = enqueue_finish(m, false);
    if (rc) return rc;
  }
  // the slice's sampled sources are all appended (after the partitioned
  // scan's partition kernel, so the sort runs beside its marking and
  // stamping; else after the scans): the pipeline stream may sort them
  if (!m->overlap_report && !m->hold_scans) {
    if (m->sampled_pending) {
      m->ev_sort = m->ev_sampled;
    } else {
      HIP_TRY(m, hipEventRecord(m->ev_scanned, m->stream));
      m->ev_sort = m->ev_scanned;
    }
  }
  m->sampled_pending = false;
  if (m->overlap_report ? m->slice >= 2 : (m->discrete && m->slice >= 1))
    HIP_TRY(m, wait_unless_done(m->stream, m->ev_done[m->overlap_report ? p : p ^ 1]));
  // with graphs, each phase is timed as a whole: the first as the sweeps
  // (with the candidate work when the report copy overlaps the next scans),
  // the second as the estimate (as the report copy when it overlaps)
  hipEvent_t ta;
  int rc = SRLA_OK;
  if (m->hold_scans && !m->timing) {
    // the scans wait for the report anyway: the sort follows them on their
    // stream, where it neither waits for an event nor queues behind the
    // previous slice's carried list on the pipeline stream; with the
    // snapshot in the same launch
    rc = run_phase(m, PH_SORT_SNAPSHOT, (int)(m->slice % kCycle), m->stream);
    if (rc) return rc;
  } else {
    if (m->hold_scans) {
      if (m->use_graph) span_begin(m, m->stream, &ta);
      rc = run_phase(m, PH_SORT, (int)(m->slice % kCycle), m->stream);
      if (rc) return rc;
      if (m->use_graph) span_end(m, m->stream, ST_FINALIZE, ta);
    }
    if (m->use_graph) span_begin(m, m->stream, &ta);
    rc = run_phase(m, PH_SNAPSHOT, (int)(m->slice % kCycle), m->stream);
    if (rc) return rc;
    if (m->use_graph) span_end(m, m->stream, m->overlap_report ? ST_ESTIMATE : ST_SWEEP, ta);
  }
  if (!m->hold_scans) HIP_TRY(m, hipEventRecord(m->ev_snap, m->stream));
  // the next slice's scans reuse the sampled-source list and count of the
  // previous slice's parity: they wait for its second phase (with held
  // scans this slice's candidate work, next on this stream, needs it too:
  // Algorithm 3's carried list and SI counters of the previous slice)
  if (!m->overlap_report && !m->discrete && m->slice >= 1)
    HIP_TRY(m, wait_unless_done(m->stream, m->ev_done[p ^ 1]));
  m->n_pending++;
  m->slice++;
  m->slice_pairs[m->slice & 1] = 0;
  // with overlap_report the second phase waits for the next slice's first
  // scan (or for srla_wait_report, whichever comes first)
  if (m->overlap_report) {
    m->finish_deferred = true;
    return SRLA_OK;
  }
  return enqueue_finish(m, false);
}

int srla_wait_report(srla_monitor_t* m, srla_report_t* out) {
  if (!m || !out) return m ? fail(m, SRLA_E_INVAL, "out is NULL") : SRLA_E_INVAL;
  if (m->poisoned) return fail(m, SRLA_E_STATE, "monitor is poisoned by an earlier error");
  if (!m->n_pending) return fail(m, SRLA_E_STATE, "no closed slice is waiting");
  // the oldest closed slice whose report is not collected yet: its parity
  // (events) and its report set
  const uint64_t e_slice = m->slice - m->n_pending;
  const int pe = (int)(e_slice & 1), q = (int)(e_slice % kSets);
  if (m->finish_deferred && m->n_pending == 1) {
    const int rc = enqueue_finish(m, false);
    if (rc) return rc;
  }
  // the report is complete once it is published; the carried list and SI
  // (ev_done) may still be in progress behind it
  HIP_TRY(m, hipEventSynchronize(m->ev_pub[pe]));
  m->n_pending--;
  const HostStatus& hs = *m->h_status[q];
  const Counters c = hs.cnt;
  if (c.overflow) {
    m->poisoned = true;
    collect_spans(m, false);
    return fail(m, SRLA_E_CAPACITY, "candidate list exceeds max_candidates");
  }
  if (m->timed[pe]) m->estimates++;
  collect_spans(m, false);
  const Geo& geo = m->geo;
  for (uint32_t i = 0; i < geo.u; ++i) m->h_row_fill64[q][i] = hs.row_fill[i];
  out->slice = hs.slice;
  out->window_full = hs.slice >= (uint64_t)(geo.k - 1) ? 1u : 0u;
  out->n = c.n_cand;
  out->ip = m->h_ip[q];
  out->est = m->h_est[q];
  out->flags = m->h_flags[q];
  out->union_weight = m->h_U[q];
  out->re_weight = m->h_W[q];
  out->row_fill = m->h_row_fill64[q];
  out->up = hs.up;
  out->n_touched = c.n_unique;
  out->n_new = c.n_new;
  out->latency_ms = m->clock_khz > 0 && hs.t_done >= hs.t_close
                        ? (double)(hs.t_done - hs.t_close) / (double)m->clock_khz
                        : 0.0;
  out->host_bytes = hs.host_bytes;
  return SRLA_OK;
}

int srla_estimate(srla_monitor_t* m, srla_report_t* out) {
  if (!m || !out) return m ? fail(m, SRLA_E_INVAL, "out is NULL") : SRLA_E_INVAL;
  if (m->n_pending)
    return fail(m, SRLA_E_STATE, "an earlier closed slice's report has not been collected");
  const int rc = srla_close_slice(m);
  if (rc) return rc;
  return srla_wait_report(m, out);
}

int srla_dump_state(srla_monitor_t* m, int which, uint16_t* host_out, uint64_t cells) {
  if (!m || !host_out) return m ? fail(m, SRLA_E_INVAL, "host_out is NULL") : SRLA_E_INVAL;
  HIP_TRY(m, hipStreamSynchronize(m->stream));
  HIP_TRY(m, hipStreamSynchronize(m->pipe_use));
  if (which == SRLA_DUMP_SI) {
    if (cells != m->n_si) return fail(m, SRLA_E_INVAL, "cells does not match the array size");
    std::vector<uint32_t> c(16 * m->n_si);
    HIP_TRY(m, hipMemcpy(c.data(), m->si_cnt, c.size() * 4, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < m->n_si; ++i) {
      uint16_t w = 0;
      for (int b = 0; b < 16; ++b)
        if (c[16 * i + b]) w = (uint16_t)(w | (1u << b));
      host_out[i] = w;
    }
    return SRLA_OK;
  }
  if (m->discrete) {
    // a DR is one bit: distance 0 if set in the open slice, 1 if set in the
    // slice closed last, beyond the window (all ones) otherwise
    const uint64_t n = which == SRLA_DUMP_LE ? m->n_le : which == SRLA_DUMP_RE ? m->n_re : 0;
    if (!n) return fail(m, SRLA_E_INVAL, "unknown state array");
    if (cells != n) return fail(m, SRLA_E_INVAL, "cells does not match the array size");
    const int p = (int)(m->slice & 1);
    // the SRE bits sit in the even words of the interleaved activity layout
    const bool re = which == SRLA_DUMP_RE;
    uint64_t* const* bits = re ? m->rebits : m->lebits;
    const uint64_t words = (re ? 2 : 1) * bitmap_words(n);
    std::vector<uint64_t> open(words), last(words);
    HIP_TRY(m, hipMemcpy(open.data(), bits[p], words * 8, hipMemcpyDeviceToHost));
    HIP_TRY(m, hipMemcpy(last.data(), bits[p ^ 1], words * 8, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
      const uint64_t w = re ? 2 * (i >> 6) : (i >> 6);
      const bool o = (open[w] >> (i & 63)) & 1u, l = (last[w] >> (i & 63)) & 1u;
      host_out[i] = o ? 0 : (l && m->slice > 0 ? 1 : 65535);
    }
    return SRLA_OK;
  }
  const uint16_t* src;
  uint64_t n;
  if (which == SRLA_DUMP_LE) { src = m->le; n = m->n_le; }
  else if (which == SRLA_DUMP_RE) { src = m->re; n = m->n_re; }
  else return fail(m, SRLA_E_INVAL, "unknown state array");
  if (cells != n) return fail(m, SRLA_E_INVAL, "cells does not match the array size");
  HIP_TRY(m, hipMemcpy(host_out, src, n * 2, hipMemcpyDeviceToHost));
  const int32_t now = stamp_code(m->slice);
  for (uint64_t i = 0; i < n; ++i) {
    const uint16_t c = host_out[i];
    if (c == 0) { host_out[i] = 65535; continue; }
    int32_t d = now - (int32_t)c;
    if (d < 0) d += (int32_t)kStampPeriod;
    host_out[i] = d >= (int32_t)kScrubAge ? 65535 : (uint16_t)d;
  }
  return SRLA_OK;
}

int srla_set_timing(srla_monitor_t* m, int enabled) {
  if (!m) return SRLA_E_INVAL;
  m->timing = enabled != 0 && enabled != SRLA_TIMING_SCANS;
  m->time_scans = enabled == SRLA_TIMING_SCANS;
  return SRLA_OK;
}

int srla_timings(srla_monitor_t* m, srla_timings_t* out, int reset) {
  if (!m || !out) return SRLA_E_INVAL;
  HIP_TRY(m, hipStreamSynchronize(m->stream));
  HIP_TRY(m, hipStreamSynchronize(m->pipe_use));
  collect_spans(m, true);
  out->scan_ms = m->acc_ms[ST_SCAN];
  out->scan_launches = m->scan_launches;
  out->scan_pairs = m->scan_pairs;
  out->sweep_ms = m->acc_ms[ST_SWEEP];
  out->finalize_ms = m->acc_ms[ST_FINALIZE];
  out->estimate_ms = m->acc_ms[ST_ESTIMATE];
  out->slide_ms = m->acc_ms[ST_SLIDE];
  out->report_ms = m->acc_ms[ST_REPORT];
  out->estimates = m->estimates;
  if (reset) {
    for (double& x : m->acc_ms) x = 0;
    m->scan_launches = m->scan_pairs = m->estimates = 0;
  }
  return SRLA_OK;
}

// ------------------------------------------------------------------ groups

}  // extern "C"

struct srla_group {
  std::vector<srla_monitor*> mons;
  hipStream_t stream = nullptr;
  // the members' end-of-slice pipelines share one stream with a hardware
  // queue of its own: a member's if one has it, else the group's own
  hipStream_t pipe = nullptr;
  bool pipe_created = false, pipe_own = false;
  GroupMember* d_members = nullptr;
  std::vector<GroupMember> uploaded;
  uint32_t scan_blocks = 0;
  std::string err;
};

namespace {

bool same_member(const GroupMember& a, const GroupMember& b) {
  return std::memcmp(&a, &b, sizeof(GroupMember)) == 0;
}

int group_fail(srla_group* g, int code, const std::string& what) {
  if (g) g->err = what;
  return code;
}

}  // namespace

extern "C" {

int srla_group_create(srla_monitor_t* const* monitors, uint32_t n, uint32_t scan_blocks,
                      srla_group_t** out) {
  if (!out || !monitors || n < 1 || n > (uint32_t)kMaxGroup) return SRLA_E_INVAL;
  for (uint32_t i = 0; i < n; ++i) {
    if (!monitors[i] || monitors[i]->stream != monitors[0]->stream) return SRLA_E_INVAL;
    if (monitors[i]->discrete || monitors[i]->overlap_report) return SRLA_E_INVAL;
    for (uint32_t j = 0; j < i; ++j)
      if (monitors[j] == monitors[i]) return SRLA_E_INVAL;
  }
  srla_group* g = new (std::nothrow) srla_group();
  if (!g) return SRLA_E_NOMEM;
  g->mons.assign(monitors, monitors + n);
  g->stream = monitors[0]->stream;
  g->scan_blocks = scan_blocks;
  // one pipeline stream for all members: with a stream each, more streams
  // than hardware queues share queues, and a member's pipeline then waits
  // in the scan stream's queue behind the next group scan
  for (srla_monitor* m : g->mons)
    if (!g->pipe && m->pipe_own) g->pipe = m->pipe;
  if (!g->pipe) {
    if (create_queue_stream(&g->pipe, &g->pipe_own) != hipSuccess) {
      (void)hipGetLastError();
      delete g;
      return SRLA_E_DEVICE;
    }
    g->pipe_created = true;
  }
  for (srla_monitor* m : g->mons) {
    if (hipStreamSynchronize(m->pipe_use) != hipSuccess) {
      (void)hipGetLastError();
      if (g->pipe_created) destroy_queue_stream(g->pipe, g->pipe_own);
      delete g;
      return SRLA_E_DEVICE;
    }
  }
  for (srla_monitor* m : g->mons) m->pipe_use = g->pipe;
  if (hipMalloc((void**)&g->d_members, n * sizeof(GroupMember)) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return SRLA_E_NOMEM;
  }
  *out = g;
  return SRLA_OK;
}

int srla_group_scan(srla_group_t* g, const uint32_t* pairs, uint64_t n, int on_device) {
  if (!g) return SRLA_E_INVAL;
  if (n == 0) return SRLA_OK;
  if (!pairs) return group_fail(g, SRLA_E_INVAL, "pairs is NULL");
  if (!on_device) return group_fail(g, SRLA_E_INVAL, "a group scans device-resident pairs");
  GroupScanArgs args{};
  std::vector<GroupMember> table(g->mons.size());
  for (size_t i = 0; i < g->mons.size(); ++i) {
    srla_monitor* m = g->mons[i];
    if (m->poisoned) return group_fail(g, SRLA_E_STATE, "a member monitor is poisoned");
    const int p = (int)(m->slice & 1);
    const int rc = reserve_touched(m, m->slice_pairs[p] + n);
    if (rc) return group_fail(g, rc, m->err);
    GroupMember& gm = table[i];
    std::memset(&gm, 0, sizeof(gm));
    gm.geo = m->geo;
    gm.le = m->le;
    gm.re = m->re;
    gm.touched[0] = m->touched[0];
    gm.touched[1] = m->touched[1];
    gm.tcount = m->tcount;
    args.code[i] = stamp_code(m->slice);
    args.parity |= (uint64_t)p << i;
  }
  // members that all scan in partitioned form: each member's partitioned scan
  // over the pairs (the pairs are read once per member, the stores go out in
  // lines) instead of the fused kernel's random stores
  bool all_part = true;
  for (srla_monitor* m : g->mons) all_part = all_part && m->part_scan;
  if (all_part) {
    for (srla_monitor* m : g->mons) {
      const int p = (int)(m->slice & 1);
      m->sampled_pending = !m->hold_scans;
      const hipError_t e = launch_scan_partition(
          pairs, n, m->geo, stamp_code(m->slice), m->le, m->re, m->touched[p], m->tcount + p,
          m->part_entries, m->part_offs, m->part_marks, g->stream, kPartChunks, nullptr, 0,
          part_unit_of(&m->cfg), m->sampled_pending ? m->ev_sampled : nullptr);
      if (e != hipSuccess) return group_fail(g, SRLA_E_DEVICE, hipGetErrorString(e));
    }
    for (srla_monitor* m : g->mons) {
      const hipError_t e = launch_scan_end(m->ps, (uint32_t)(m->slice & 1), g->stream);
      if (e != hipSuccess) return group_fail(g, SRLA_E_DEVICE, hipGetErrorString(e));
      m->slice_pairs[m->slice & 1] += n;
      m->scan_launches++;
      m->scan_pairs += n;
    }
    return SRLA_OK;
  }
  for (srla_monitor* m : g->mons) m->sampled_pending = false;
  bool changed = g->uploaded.size() != table.size();
  for (size_t i = 0; !changed && i < table.size(); ++i)
    changed = !same_member(table[i], g->uploaded[i]);
  if (changed) {
    // the table is read by earlier fused scans still queued on the stream
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess)
      e = hipMemcpy(g->d_members, table.data(), table.size() * sizeof(GroupMember),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) return group_fail(g, SRLA_E_DEVICE, hipGetErrorString(e));
    g->uploaded = table;
  }
  const hipError_t e = launch_scan_group(pairs, n, g->d_members, (uint32_t)table.size(), args,
                                         g->scan_blocks, g->stream);
  if (e != hipSuccess) return group_fail(g, SRLA_E_DEVICE, hipGetErrorString(e));
  for (srla_monitor* m : g->mons) {
    const hipError_t e2 = launch_scan_end(m->ps, (uint32_t)(m->slice & 1), g->stream);
    if (e2 != hipSuccess) return group_fail(g, SRLA_E_DEVICE, hipGetErrorString(e2));
    m->slice_pairs[m->slice & 1] += n;
    m->scan_launches++;
    m->scan_pairs += n;
  }
  return SRLA_OK;
}

int srla_group_destroy(srla_group_t* g) {
  if (!g) return SRLA_OK;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->pipe) (void)hipStreamSynchronize(g->pipe);
  for (srla_monitor* m : g->mons) m->pipe_use = m->pipe;
  if (g->pipe_created) destroy_queue_stream(g->pipe, g->pipe_own);
  if (g->d_members) (void)hipFree(g->d_members);
  delete g;
  return SRLA_OK;
}

const char* srla_group_last_error(const srla_group_t* g) {
  if (!g) return "no group";
  return g->err.c_str();
}

int srla_destroy(srla_monitor_t* m) {
  release(m);
  return SRLA_OK;
}

const char* srla_last_error(const srla_monitor_t* m) {
  if (!m) return "no monitor";
  return m->err.c_str();
}

}  // extern "C"
