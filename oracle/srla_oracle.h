/*
 * SRLA oracle: declarations.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded CPU
 * statement of what the SRLA sliding super-point estimator computes (Sections
 * 3 and 4 of the SRLA paper, arXiv 1803.10369).  Only the test suite, the
 * smoke check and the CPU-baseline leg of the bench may load it.  It shares no
 * source with the GPU library; the two agree only because both follow the
 * same paper and the same written readings of it.
 *
 * Every distance recorder (DR) is stored as a distance, exactly as Section 3.2
 * defines it: z = 16 bits, DRinit sets all ones (65535), DRset sets 0, DRslide
 * increments below 65535, DRjoin takes the maximum, and a DR counts as
 * "in the window" iff its value is smaller than the window length k.
 */
#ifndef SRLA_ORACLE_H
#define SRLA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* number of hash functions drawn from the seed: RH_0..RH_{u-1}, H1, H2, H3, H4 */
#define ORC_MAX_U 16
#define ORC_NHASH(u) ((u) + 4)

typedef struct {
    uint32_t k;          /* window length in slices, 1..32767 */
    uint32_t theta;      /* super point threshold (Definition 2), >= 1 */
    uint32_t u;          /* SEA rows (Section 4.1), 1..16 */
    uint32_t v_re;       /* columns holding SI and SRE */
    uint32_t g;          /* DRs per SRE, 1..64 */
    uint32_t v_le;       /* columns holding LE */
    uint32_t G;          /* DRs per LE (the paper's g'), multiple of 64 */
    uint64_t hash_seed;  /* SplitMix64 seed for all hash parameters */
    uint64_t max_candidates;
    uint32_t sequential; /* 0: slice-synchronous candidate check (the reading
                            both implementations share); 1: Algorithm 2's
                            check after every sampled pair, in stream order */
} orc_config;

/* flags of one reported candidate */
#define ORC_SUPER 1u  /* estimate >= theta */
#define ORC_SAT   2u  /* Eq9 undefined (union LE full): estimate is +inf */
#define ORC_NEW   4u  /* inserted into the candidate list during this slice */
#define ORC_KEEP  8u  /* carried into the next slice's list by Algorithm 3 */

typedef struct {
    uint64_t slice;               /* index of the slice just closed */
    uint32_t window_full;         /* slice >= k-1 */
    uint64_t n;                   /* |CSIP| */
    const uint32_t *ip;           /* NCSIP of the previous slice ascending, then N_t ascending */
    const double *est;            /* Eq9 */
    const uint8_t *flags;
    const uint32_t *union_weight; /* |ULE(aip)|^k */
    const uint8_t *re_weight;     /* |URE(aip)|^k before the slide */
    const uint64_t *row_fill;     /* |LDR(i)|^k, i < u */
    double up;                    /* Eq8 */
    uint64_t n_touched;           /* distinct sources with a sampled pair */
    uint64_t n_new;
} orc_report;

typedef struct orc_monitor orc_monitor;

/* building blocks, exported so the tests can pin each one */
uint64_t orc_splitmix64_next(uint64_t *state);
uint32_t orc_lsb(uint32_t x);
uint32_t orc_tau(uint32_t theta, uint32_t g);
uint32_t orc_sre_threshold(uint32_t g);
double   orc_rho(void);
uint32_t orc_mas(uint64_t a, uint64_t b, uint32_t x);
uint32_t orc_range(uint32_t h, uint32_t m);
void     orc_hash_params(uint64_t seed, uint32_t nfun, uint64_t *a, uint64_t *b);

/* the monitor */
orc_monitor *orc_create(const orc_config *cfg);
int  orc_scan(orc_monitor *m, const uint32_t *pairs, uint64_t n);
int  orc_estimate(orc_monitor *m, orc_report *out);
int  orc_dump(const orc_monitor *m, int which, uint16_t *out, uint64_t cells);
uint64_t orc_slice(const orc_monitor *m);
void orc_destroy(orc_monitor *m);

#ifdef __cplusplus
}
#endif
#endif
