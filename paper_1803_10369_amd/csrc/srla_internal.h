// Internal declarations of the gfx950 SRLA library: the per-monitor constant
// block that every kernel receives by value, the device-side hash and stamp
// helpers, and the launchers the host runtime calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srla {

constexpr int kMaxU = 16;
// partial sums per row of the LE sweep's row fills (blocks add to slot
// block mod kFillSlots)
constexpr uint32_t kFillSlots = 32;
constexpr int kWave = 64;
constexpr int kBlock = 256;

// DR cells hold slice stamps instead of distances: 0 = never set (or scrubbed),
// otherwise code(s) = (s mod 65535) + 1 of the last slice s that set the cell.
// At open slice t the cell's distance (Section 3.2) is
// (code(t) - cell) mod 65535, so DRslide is free and DRset is one plain store.
// Stamps whose distance reaches kScrubAge are zeroed before they can alias.
constexpr uint32_t kStampPeriod = 65535;
constexpr uint32_t kScrubAge = 32768;

__host__ __device__ inline uint16_t stamp_code(uint64_t slice) {
  return (uint16_t)(slice % kStampPeriod + 1);
}

// Hash function of the multiply-add-shift family:
// h(x) = ((a*x + b) mod 2^64) >> 32.
struct HashFn {
  uint64_t a, b;
};

// Everything a kernel needs to know about one monitor.
struct Geo {
  uint32_t u, v_re, g, v_le, G;  // G = g' (DRs per LE)
  uint32_t k;                    // window in slices
  uint32_t theta;
  uint32_t tau_mask;             // LSB(h) >= tau  <=>  (h & tau_mask) == 0
  uint32_t t_re;                 // ceil(rho * g)
  uint32_t words;                // G / 64 bitmap words per LE
  HashFn rh[kMaxU];              // RH_0 .. RH_{u-1}
  HashFn h1, h2, h3, h4;
};

__device__ __forceinline__ uint32_t mas(const HashFn& f, uint32_t x) {
  return (uint32_t)((f.a * (uint64_t)x + f.b) >> 32);
}

// maps a 32-bit hash to [0, m)
__device__ __forceinline__ uint32_t hrange(uint32_t h, uint32_t m) {
  return (uint32_t)(((uint64_t)h * (uint64_t)m) >> 32);
}

// distance of a nonzero stamp at open-slice code `now`
__device__ __forceinline__ uint32_t stamp_age(uint32_t now, uint32_t cell) {
  int32_t d = (int32_t)now - (int32_t)cell;
  return (uint32_t)(d < 0 ? d + (int32_t)kStampPeriod : d);
}

// "DR < k": set inside the window that ends at the slice whose code is `now`
__device__ __forceinline__ bool in_window(uint32_t now, uint32_t cell, uint32_t k) {
  return cell != 0 && stamp_age(now, cell) < k;
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Device counters of one slice's end-of-slice pipeline.
struct Counters {
  uint32_t touched;      // sampled-source appends of the slice (copied in)
  uint32_t n_unique;     // distinct sampled sources
  uint32_t n_new;        // new candidates N_t
  uint32_t n_cand;       // |CSIP_t| (clamped to capacity)
  uint32_t n_keep;       // |NCSIP_t|
  uint32_t overflow;     // CSIP_t exceeded capacity
  uint32_t n_keep_a;     // carried candidates of CSIP_t that stay in NCSIP_t
  uint32_t pad;
};

constexpr uint32_t kEndSlots = 64;

// Device-resident state the end-of-slice pipeline reads instead of host
// arguments, so one recorded pipeline serves every slice of a parity.
struct PipeState {
  uint32_t now;          // stamp code of the slice whose candidate work is next
  uint32_t n_ncsip;      // |NCSIP| carried into it
  uint64_t slice;        // its index
  uint64_t t_close[2];   // device wall clock when the last closed slice of each
                         // parity ended: its last scan finished (or, for a slice
                         // without scans, its end-of-slice work began)
  uint64_t t_scan[2];    // device wall clock at the end of the last scan of the
                         // open slice of each parity (scans with a marker kernel)
  uint32_t scanned[2];   // that slice has had a scan
  uint32_t snap;         // stamp code of the slice snapshotted last (0: none yet);
                         // the snapshot keeps its own count so that it need not
                         // wait for the previous slice's candidate work
  uint32_t pad;
  uint32_t snap_code[2]; // the same for the sweep of the stamp arrays, by the
                         // parity of the slice snapshotted (the sweep of parity
                         // p reads the code of p ^ 1 and writes that of p)
  // the partitioned scan's last kernel: each workgroup raises slot
  // blockIdx % kEndSlots to the clock when it is done (few workgroups per
  // slot, so the atomics do not queue on one address); the end of the scan
  // is the largest slot
  unsigned long long t_end[2][kEndSlots];
  // bytes the estimate wrote into the host report arrays, in slots by
  // workgroup (summed and cleared when the report is published)
  unsigned long long rep_bytes[kEndSlots];
};

// Pinned host block the status kernel fills at the end of every slice.
struct HostStatus {
  Counters cnt;
  double up;
  unsigned long long row_fill[kMaxU];
  uint64_t slice;
  uint64_t t_close;      // device wall clock: the slice's last scan ended
  uint64_t t_done;       //   and the report was complete in host memory
  uint64_t host_bytes;   // bytes the estimate wrote into the report arrays
};

// Report arrays in pinned host memory, as device-visible pointers.  With
// mir_est / mir_flags (device copies of what the host arrays of this set
// hold), the estimate writes into host memory only the 16-byte pieces whose
// contents change.
struct ReportPtrs {
  uint32_t* ip;
  double* est;
  uint8_t* flags;
  uint32_t* U;
  uint8_t* W;
  double* mir_est;
  uint8_t* mir_flags;
};

// One member of a monitor group, as the fused scan kernel sees it.
struct GroupMember {
  Geo geo;
  uint16_t* le;
  uint16_t* re;
  uint32_t* touched[2];   // sampled sources, by slice parity
  uint32_t* tcount;       // [2] their counts
};

constexpr int kMaxGroup = 64;

// Per-launch arguments of the fused scan: each member's stamp code and slice
// parity (members may be at different slices).
struct GroupScanArgs {
  uint16_t code[kMaxGroup];
  uint64_t parity;        // bit m = parity of member m's open slice
};

// Fixed grids of the end-of-slice kernels (they loop over device counts).
constexpr uint32_t kPipeBlocks = 1024;

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return the launch status.

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t st);

// Algorithm 2 for n pairs of the open slice (stamp code `code`); sampled
// sources are appended to `touched`, counted in *tcount.  max_blocks caps
// the grid (0: one block per tile of pairs).  claim: two device words, zero
// at first use, for the flat form's tile claims; *slot (host) selects the
// one a launch uses and is flipped by every launch of that form.  Launches
// that share claim must be ordered (one stream).  mark != 0 (n > 0): *started
// is set to mark as the scan starts (by the scan kernel itself, or by a
// marker kernel just before it).
hipError_t launch_scan(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                       uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                       uint32_t* claim, uint32_t* slot, bool xcd_aware, uint32_t max_blocks,
                       hipStream_t st, uint32_t* started = nullptr, uint32_t mark = 0);

// Algorithm 2 of every member of a group for n pairs, each pair loaded once
hipError_t launch_scan_group(const uint32_t* pairs, uint64_t n, const GroupMember* members,
                             uint32_t n_members, const GroupScanArgs& args, uint32_t max_blocks,
                             hipStream_t st);

// The snapshot in one launch (slice parity p): the slice's close (the end of
// its scans, its stamp code), |LDR(i)|^k by row into kFillSlots partial sums
// per row (fill_part, u x kFillSlots, zero beforehand; the fold clears it
// again), the LE
// activity bitmap and scrub; the SRE activity maps (inside the window now /
// after the slide) and scrub
hipError_t launch_sweep(uint16_t* le, uint64_t* bitmap, unsigned long long* fill_part,
                        uint16_t* re, uint64_t n_re, uint64_t* act, const Geo& geo,
                        PipeState* ps, uint32_t p, hipStream_t st);

// keys-only ascending sort of *n_dev uint32 keys, in place (tmp is scratch of
// at least *n_dev words); aux: sort_aux_words() words, zero before the first
// sort (each sort leaves them so).
uint64_t sort_aux_words();
hipError_t sort_u32(uint32_t* keys, uint32_t* tmp, const uint32_t* n_dev, uint32_t* aux,
                    hipStream_t st);

// exclusive-scan helper storage for compaction of up to n elements
uint64_t compact_block_words(uint64_t n);

// stable compaction of vals[i] with (flags[i] & mask) != 0, i < *n_dev
// (n_dev <= n_max); result count -> *out_count
hipError_t compact_u32(const uint8_t* flags, uint8_t mask, const uint32_t* vals,
                       const uint32_t* n_dev, uint64_t n_max, uint32_t* out,
                       uint32_t* out_count, uint32_t* block_words, hipStream_t st);

// (with fill_part: its first block folds the sweep's partial sums into
// row_fill and evaluates Eq8 into *up first)
hipError_t launch_finalize(const uint32_t* sorted, const uint32_t* n_dev, const uint64_t* act,
                           const uint32_t* si_cnt, const Geo& geo, uint8_t* mark, Counters* cnt,
                           const unsigned long long* fill_part, unsigned long long* row_fill,
                           double* up, hipStream_t st);

// CSIP_t = the carried list (the first ps->n_ncsip entries of cand) followed
// by the cnt->n_new new candidates, appended to cand (capacity cap)
hipError_t launch_join(const PipeState* ps, const uint32_t* news, Counters* cnt, uint64_t cap,
                       uint32_t* cand, hipStream_t st);
// cnt->n_keep_a += KEEP flags among the carried part of CSIP_t
hipError_t launch_count_keep(const uint8_t* cflags, const PipeState* ps, Counters* cnt,
                             hipStream_t st);
// merges the ascending runs [0, *na) and [*na, *n) of in into out
hipError_t launch_merge_runs(const uint32_t* in, const uint32_t* na, const uint32_t* n,
                             uint32_t* out, hipStream_t st);
// copies *n uint32 from src (device) to dst (pinned host memory, 16-byte aligned)
hipError_t launch_ip_precopy(const uint32_t* src, const uint32_t* n, uint32_t* dst,
                             hipStream_t st);

hipError_t launch_union_prob(const unsigned long long* row_fill, const Geo& geo,
                             double* up, hipStream_t st);

// Eq9 for every candidate of CSIP (csip: the carried list, ps->n_ncsip
// entries, then the new candidates); rows whose row fill is g' * v_le (every
// LE DR inside the window) are not gathered.  skip_carried_ip: the report's
// ip array holds the carried list already, only the new candidates' are
// written
hipError_t launch_estimate(const uint32_t* csip, const Counters* cnt, const PipeState* ps,
                           bool skip_carried_ip, const uint64_t* bitmap,
                           const uint64_t* act, const double* up,
                           const unsigned long long* row_fill, const Geo& geo, uint8_t* cflags,
                           const ReportPtrs& out, hipStream_t st);

// copies the first *n report entries from device staging arrays to the host
// arrays (U and W only where `to` has them); with expect != 0, only once
// *started == expect (a bounded wait)
hipError_t launch_report_copy(const uint32_t* n, const ReportPtrs& from, const ReportPtrs& to,
                              const uint32_t* started, uint32_t expect, hipStream_t st);
// sets *started = value: the scan enqueued behind it on the stream is about to start
hipError_t launch_mark_scan(uint32_t* started, uint32_t value, hipStream_t st);

// Algorithm 3's SI step on the per-bit counters (after the KEEP flags are final)
hipError_t launch_si_update(const uint32_t* csip, const uint8_t* cflags, const Counters* cnt,
                            uint32_t* si_cnt, const Geo& geo, hipStream_t st);

// records the device wall clock at the end of a scan of the open slice of
// parity p
hipError_t launch_scan_end(PipeState* ps, uint32_t p, hipStream_t st);
// takes the end of the last scan of the closing slice of parity p (or, without
// scans, the device wall clock now) as the slice's end, advances the
// snapshot's stamp code and clears n_clear words of the row-fill sums
hipError_t launch_begin_close(PipeState* ps, unsigned long long* row_fill, uint32_t n_clear,
                              uint32_t p, hipStream_t st);
// records the device wall clock once the report is complete in host memory
hipError_t launch_mark_done(HostStatus* out, hipStream_t st);
// publishes the slice's counters, Eq8 and row fills to the host (and the
// candidate count to *report_n), carries |NCSIP| into the state, advances the
// state to the next slice, and clears the slice's counters (and the
// sampled-source count of its parity)
hipError_t launch_status(Counters* cnt, uint32_t* tcount, const double* up,
                         const unsigned long long* row_fill, uint32_t u, PipeState* ps,
                         uint32_t p, HostStatus* out, uint32_t* report_n, hipStream_t st);
// the two halves of launch_status (report_n not written): publish copies the
// slice's counters, Eq8 and row fills into the host block and reads the
// clock (the report is complete); advance carries |NCSIP| into the state,
// moves it to the next slice and clears the counters, once Algorithm 3's
// carried list is final
hipError_t launch_publish(const Counters* cnt, const uint32_t* tcount, const double* up,
                          const unsigned long long* row_fill, uint32_t u, PipeState* ps,
                          uint32_t p, HostStatus* out, hipStream_t st);
hipError_t launch_advance(Counters* cnt, uint32_t* tcount, PipeState* ps, hipStream_t st);

}  // namespace srla
