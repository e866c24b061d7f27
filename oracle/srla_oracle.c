/*
 * SRLA oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded C statement of the SRLA method of arXiv 1803.10369:
 * the distance recorder DR (Section 3.2), the sliding rough estimator SRE
 * (Section 3.2, Eq1), the sliding linear estimator SLE (Section 3.3, Eq6-Eq7),
 * and the SE array SEA with UnionSE (Algorithm 1), ScanIPpair (Algorithm 2),
 * the noise-corrected union estimate (Eq8-Eq9) and the update before sliding
 * (Algorithm 3), all in Section 4.
 *
 * Nothing here is blocked, fused or reordered: every DR is a distance, every
 * slide touches every DR, every union walks all u rows.  Readings of points
 * the paper leaves open are stated where they are used:
 *
 *  hash family   The paper names Indyk's min-wise family for H1 and only the
 *                ranges of the others.  Reading: every hash is Dietzfelbinger's
 *                multiply-add-shift h(x) = ((a*x + b) mod 2^64) >> 32 with
 *                64-bit (a, b), reduced to [0, m) by (h*m) >> 32.  The (a, b)
 *                of function f are outputs 2f and 2f+1 of SplitMix64 started
 *                at the hash seed, in the order RH_0..RH_{u-1}, H1, H2, H3, H4.
 *  SRE sampling  A pair updates the SRE iff LSB(H1(bip)) >= tau (Section 3.2
 *                text and the Binomial(|OP|, 2^-tau) analysis), LSB(0) = 32.
 *  LE index      H3(bip) reduced to [0, g') (Section 3.3); SI bit H4(aip) in
 *                [0, 16) (Section 4.1).
 *  detection     |URE|^k >= rho*g, i.e. >= ceil(rho*g) (Section 3.2, Alg. 3).
 *  candidates    Slice-synchronous: at the end of slice t every source with at
 *                least one sampled pair in t is checked once against the
 *                end-of-slice SRE and against SI as Algorithm 3 left it; the
 *                candidate list CSIP_t = NCSIP_{t-1} + N_t (Algorithms 2-3) is
 *                reported as the carried list, ascending, followed by the
 *                new candidates, ascending.  (With
 *                cfg.sequential the check runs after every sampled pair in
 *                stream order instead, inserting and marking SI at once --
 *                Algorithm 2 taken literally; used to measure the reading.)
 *  union DRs     Algorithm 1 starts the union SRE/LE DRs at 2^z-1 and joins
 *                with max, which would leave them at 2^z-1; the union DR is
 *                read as the max over the u rows (the join's identity is 0).
 *  geometry      SI/SRE columns (v_re) and LE columns (v_le) may differ; the
 *                row hash RH_i is shared, so v_re == v_le is the paper's SE.
 *  Eq9 edges     UP == 1 or 1 - x <= 0 gives +inf with the SAT flag; negative
 *                estimates are reported as computed.
 */
#include "srla_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define DR_MAX 65535u   /* 2^z - 1 with z = 16 (Section 3.2) */

struct orc_monitor {
    orc_config cfg;
    uint32_t tau;      /* Eq1 */
    uint32_t t_re;     /* ceil(rho * g) */
    uint64_t ha[ORC_NHASH(ORC_MAX_U)];
    uint64_t hb[ORC_NHASH(ORC_MAX_U)];
    uint16_t *RE;      /* [u][v_re][g] distances */
    uint16_t *LE;      /* [u][v_le][G] distances */
    uint16_t *SI;      /* [u][v_re] 16-bit super point indicators */
    uint64_t slice;    /* index of the open slice */
    int poisoned;

    uint32_t *touched; uint64_t n_touched, cap_touched;
    uint32_t *seq_new; uint64_t n_seq_new, cap_seq_new;   /* sequential mode's N_t */
    uint32_t *ncsip;   uint64_t n_ncsip;          /* ascending */

    /* report storage, valid until the next estimate */
    uint32_t *r_ip; double *r_est; uint8_t *r_flags;
    uint32_t *r_U; uint8_t *r_W; uint64_t r_cap;
    uint64_t row_fill[ORC_MAX_U];
};

/* ---------------------------------------------------------------- hashing */

uint64_t orc_splitmix64_next(uint64_t *state)
{
    /* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) */
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ull;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_hash_params(uint64_t seed, uint32_t nfun, uint64_t *a, uint64_t *b)
{
    uint64_t s = seed;
    uint32_t f;
    for (f = 0; f < nfun; f++) {
        a[f] = orc_splitmix64_next(&s);
        b[f] = orc_splitmix64_next(&s);
    }
}

uint32_t orc_mas(uint64_t a, uint64_t b, uint32_t x)
{
    uint64_t v = a * (uint64_t)x + b;   /* mod 2^64 by unsigned wrap-around */
    return (uint32_t)(v >> 32);
}

uint32_t orc_range(uint32_t h, uint32_t m)
{
    return (uint32_t)(((uint64_t)h * (uint64_t)m) >> 32);
}

/* Definition 4: index of the first 1 bit counted from the right. */
uint32_t orc_lsb(uint32_t x)
{
    uint32_t i;
    if (x == 0) return 32;
    for (i = 0; i < 32; i++)
        if ((x >> i) & 1u) return i;
    return 32;
}

/* Eq1: tau = ceil(log2(theta / g)), as the smallest tau >= 0 with g*2^tau >= theta */
uint32_t orc_tau(uint32_t theta, uint32_t g)
{
    uint32_t tau = 0;
    while ((uint64_t)g << tau < (uint64_t)theta) tau++;
    return tau;
}

/* rho = 0.99 * (1 - e^(-1/3)) (Section 3.2, from Kane, Nelson and Woodruff) */
double orc_rho(void)
{
    return 0.99 * (1.0 - exp(-1.0 / 3.0));
}

/* the integer form of "|SRE|^k >= rho * g" */
uint32_t orc_sre_threshold(uint32_t g)
{
    return (uint32_t)ceil(orc_rho() * (double)g);
}

/* hash helpers of one monitor, in the function order of the seed expansion */
static uint32_t row_hash(const orc_monitor *m, uint32_t i, uint32_t aip)
{
    return orc_mas(m->ha[i], m->hb[i], aip);                 /* RH_i */
}
static uint32_t H1(const orc_monitor *m, uint32_t bip)
{
    uint32_t f = m->cfg.u;
    return orc_mas(m->ha[f], m->hb[f], bip);
}
static uint32_t H2(const orc_monitor *m, uint32_t bip)
{
    uint32_t f = m->cfg.u + 1;
    return orc_range(orc_mas(m->ha[f], m->hb[f], bip), m->cfg.g);
}
static uint32_t H3(const orc_monitor *m, uint32_t bip)
{
    uint32_t f = m->cfg.u + 2;
    return orc_range(orc_mas(m->ha[f], m->hb[f], bip), m->cfg.G);
}
static uint32_t H4(const orc_monitor *m, uint32_t aip)
{
    uint32_t f = m->cfg.u + 3;
    return orc_range(orc_mas(m->ha[f], m->hb[f], aip), 16);
}
static uint32_t col_re(const orc_monitor *m, uint32_t i, uint32_t aip)
{
    return orc_range(row_hash(m, i, aip), m->cfg.v_re);
}
static uint32_t col_le(const orc_monitor *m, uint32_t i, uint32_t aip)
{
    return orc_range(row_hash(m, i, aip), m->cfg.v_le);
}

/* DR cells of the SE in row i, column c */
static uint16_t *RE_dr(const orc_monitor *m, uint32_t i, uint32_t c)
{
    return m->RE + ((uint64_t)i * m->cfg.v_re + c) * m->cfg.g;
}
static uint16_t *LE_dr(const orc_monitor *m, uint32_t i, uint32_t c)
{
    return m->LE + ((uint64_t)i * m->cfg.v_le + c) * m->cfg.G;
}
static uint16_t *SI_of(const orc_monitor *m, uint32_t i, uint32_t c)
{
    return m->SI + (uint64_t)i * m->cfg.v_re + c;
}

/* ------------------------------------------------------- DR operations */

static void DRinit(uint16_t *dr) { *dr = (uint16_t)DR_MAX; }
static void DRset(uint16_t *dr) { *dr = 0; }
static void DRslide(uint16_t *dr) { if (*dr < DR_MAX) *dr = (uint16_t)(*dr + 1); }
static uint16_t DRjoin(uint16_t a, uint16_t b) { return a > b ? a : b; }

/* ---------------------------------------------------------- lifecycle */

orc_monitor *orc_create(const orc_config *cfg)
{
    orc_monitor *m;
    uint64_t n_re, n_le, n_si, x;
    if (!cfg) return NULL;
    if (cfg->u < 1 || cfg->u > ORC_MAX_U || cfg->g < 1 || cfg->g > 64 ||
        cfg->G < 64 || cfg->G % 64 != 0 || cfg->v_re < 1 || cfg->v_le < 1 ||
        cfg->k < 1 || cfg->k > 32767 || cfg->theta < 1)
        return NULL;
    m = (orc_monitor *)calloc(1, sizeof(*m));
    if (!m) return NULL;
    m->cfg = *cfg;
    m->tau = orc_tau(cfg->theta, cfg->g);
    m->t_re = orc_sre_threshold(cfg->g);
    orc_hash_params(cfg->hash_seed, ORC_NHASH(cfg->u), m->ha, m->hb);
    n_re = (uint64_t)cfg->u * cfg->v_re * cfg->g;
    n_le = (uint64_t)cfg->u * cfg->v_le * cfg->G;
    n_si = (uint64_t)cfg->u * cfg->v_re;
    m->RE = (uint16_t *)malloc(n_re * sizeof(uint16_t));
    m->LE = (uint16_t *)malloc(n_le * sizeof(uint16_t));
    m->SI = (uint16_t *)calloc(n_si, sizeof(uint16_t));
    if (!m->RE || !m->LE || !m->SI) { orc_destroy(m); return NULL; }
    for (x = 0; x < n_re; x++) DRinit(&m->RE[x]);
    for (x = 0; x < n_le; x++) DRinit(&m->LE[x]);
    return m;
}

void orc_destroy(orc_monitor *m)
{
    if (!m) return;
    free(m->RE); free(m->LE); free(m->SI);
    free(m->touched); free(m->ncsip); free(m->seq_new);
    free(m->r_ip); free(m->r_est); free(m->r_flags); free(m->r_U); free(m->r_W);
    free(m);
}

uint64_t orc_slice(const orc_monitor *m) { return m->slice; }

/* ---------------------------------------------- Algorithm 2: ScanIPpair */

static uint32_t union_re_weight(const orc_monitor *m, uint32_t aip);
static uint16_t union_si(const orc_monitor *m, uint32_t aip);
static void set_si_bits(orc_monitor *m, uint32_t aip);

static int scan_pair(orc_monitor *m, uint32_t aip, uint32_t bip)
{
    uint32_t i, leidx, reidx;

    /* every pair sets one DR of the LE in each of the u rows */
    leidx = H3(m, bip);
    for (i = 0; i < m->cfg.u; i++)
        DRset(&LE_dr(m, i, col_le(m, i, aip))[leidx]);

    /* only pairs with LSB(H1(bip)) >= tau reach the SRE */
    if (orc_lsb(H1(m, bip)) < m->tau)
        return 0;

    reidx = H2(m, bip);
    for (i = 0; i < m->cfg.u; i++)
        DRset(&RE_dr(m, i, col_re(m, i, aip))[reidx]);

    /* Algorithm 2 taken literally: check the host right away */
    if (m->cfg.sequential && union_re_weight(m, aip) >= m->t_re &&
        ((union_si(m, aip) >> H4(m, aip)) & 1u) == 0) {
        if (m->n_seq_new == m->cap_seq_new) {
            uint64_t nc = m->cap_seq_new ? 2 * m->cap_seq_new : 1024;
            uint32_t *p = (uint32_t *)realloc(m->seq_new, nc * sizeof(uint32_t));
            if (!p) return -2;
            m->seq_new = p; m->cap_seq_new = nc;
        }
        m->seq_new[m->n_seq_new++] = aip;
        set_si_bits(m, aip);
    }

    /* the candidate check runs at the end of the slice (slice-synchronous
       reading); remember that aip was sampled in this slice */
    if (m->n_touched == m->cap_touched) {
        uint64_t nc = m->cap_touched ? 2 * m->cap_touched : 1024;
        uint32_t *p = (uint32_t *)realloc(m->touched, nc * sizeof(uint32_t));
        if (!p) return -2;
        m->touched = p; m->cap_touched = nc;
    }
    m->touched[m->n_touched++] = aip;
    return 0;
}

int orc_scan(orc_monitor *m, const uint32_t *pairs, uint64_t n)
{
    uint64_t j;
    int rc;
    if (!m) return -1;
    if (m->poisoned) return -4;
    for (j = 0; j < n; j++) {
        rc = scan_pair(m, pairs[2 * j], pairs[2 * j + 1]);
        if (rc) return rc;
    }
    return 0;
}

/* --------------------------------------------- Algorithm 1: UnionSE parts */

/* |URE(aip)|^k: DRs of the union SRE (DRjoin over the u rows) below k */
static uint32_t union_re_weight(const orc_monitor *m, uint32_t aip)
{
    uint32_t i, j, w = 0;
    for (j = 0; j < m->cfg.g; j++) {
        /* Algorithm 1 starts URE at 2^z-1, but under DRjoin = max that value
           would absorb every row; the join is started from row 0 instead,
           which is the max over the u rows */
        uint16_t ure = RE_dr(m, 0, col_re(m, 0, aip))[j];
        for (i = 1; i < m->cfg.u; i++)
            ure = DRjoin(ure, RE_dr(m, i, col_re(m, i, aip))[j]);
        if (ure < m->cfg.k) w++;
    }
    return w;
}

/* USI(aip): AND of the u SI words */
static uint16_t union_si(const orc_monitor *m, uint32_t aip)
{
    uint32_t i;
    uint16_t usi = 0xFFFFu;
    for (i = 0; i < m->cfg.u; i++)
        usi = (uint16_t)(usi & *SI_of(m, i, col_re(m, i, aip)));
    return usi;
}

/* |ULE(aip)|^k, with the same row-0 start as the union SRE */
static uint32_t union_le_weight(const orc_monitor *m, uint32_t aip)
{
    uint32_t i, j, w = 0;
    for (j = 0; j < m->cfg.G; j++) {
        uint16_t ule = LE_dr(m, 0, col_le(m, 0, aip))[j];
        for (i = 1; i < m->cfg.u; i++)
            ule = DRjoin(ule, LE_dr(m, i, col_le(m, i, aip))[j]);
        if (ule < m->cfg.k) w++;
    }
    return w;
}

static void set_si_bits(orc_monitor *m, uint32_t aip)
{
    uint32_t i, siidx = H4(m, aip);
    for (i = 0; i < m->cfg.u; i++)
        *SI_of(m, i, col_re(m, i, aip)) |= (uint16_t)(1u << siidx);
}

static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return (a > b) - (a < b);
}

static int reserve_report(orc_monitor *m, uint64_t n)
{
    if (n <= m->r_cap) return 0;
    free(m->r_ip); free(m->r_est); free(m->r_flags); free(m->r_U); free(m->r_W);
    m->r_ip = (uint32_t *)malloc(n * sizeof(uint32_t));
    m->r_est = (double *)malloc(n * sizeof(double));
    m->r_flags = (uint8_t *)malloc(n);
    m->r_U = (uint32_t *)malloc(n * sizeof(uint32_t));
    m->r_W = (uint8_t *)malloc(n);
    m->r_cap = n;
    if (!m->r_ip || !m->r_est || !m->r_flags || !m->r_U || !m->r_W) {
        m->r_cap = 0;
        return -2;
    }
    return 0;
}

/* ------------------------------------------ end of slice: Eq8, Eq9, Alg. 3 */

int orc_estimate(orc_monitor *m, orc_report *out)
{
    const uint32_t u = m ? m->cfg.u : 0;
    uint32_t *uniq = NULL, *news = NULL, *csip = NULL;
    uint64_t n_uniq = 0, n_new = 0, n, x, j;
    uint32_t i;
    double up, G, v_le;
    int rc = 0;

    if (!m || !out) return -1;
    if (m->poisoned) return -4;

    /* distinct sources sampled in this slice */
    if (m->n_touched) {
        uniq = (uint32_t *)malloc(m->n_touched * sizeof(uint32_t));
        news = (uint32_t *)malloc(m->n_touched * sizeof(uint32_t));
        if (!uniq || !news) { rc = -2; goto done; }
        memcpy(uniq, m->touched, m->n_touched * sizeof(uint32_t));
        qsort(uniq, m->n_touched, sizeof(uint32_t), cmp_u32);
        for (x = 0; x < m->n_touched; x++)
            if (x == 0 || uniq[x] != uniq[x - 1]) uniq[n_uniq++] = uniq[x];
    }

    /* Algorithm 2's candidate check: super by the union SRE, and its own SI
       bit still clear in the union SI left by the previous Algorithm 3 */
    if (m->cfg.sequential) {
        /* already checked pair by pair; each host was inserted once (its own
           SI bits were set at insertion) */
        if (m->n_seq_new > m->n_touched) { rc = -2; goto done; }
        for (x = 0; x < m->n_seq_new; x++) news[n_new++] = m->seq_new[x];
        if (n_new) qsort(news, n_new, sizeof(uint32_t), cmp_u32);
    } else {
        for (x = 0; x < n_uniq; x++) {
            uint32_t aip = uniq[x];
            if (union_re_weight(m, aip) >= m->t_re &&
                ((union_si(m, aip) >> H4(m, aip)) & 1u) == 0)
                news[n_new++] = aip;
        }
    }

    /* CSIP of this slice: the carried list, then the new candidates (each
       ascending; the two sets are disjoint, since a carried candidate's own
       SI bit is set) */
    n = m->n_ncsip + n_new;
    if (n > m->cfg.max_candidates) { m->poisoned = 1; rc = -3; goto done; }
    if (reserve_report(m, n ? n : 1)) { rc = -2; goto done; }
    csip = m->r_ip;
    for (x = 0; x < m->n_ncsip; x++) csip[x] = m->ncsip[x];
    for (x = 0; x < n_new; x++) csip[m->n_ncsip + x] = news[x];

    /* insertion marks the candidate's SI bit in every row */
    for (x = 0; x < n_new; x++) set_si_bits(m, news[x]);

    /* |LDR(i)|^k: every LE DR of row i below k */
    for (i = 0; i < u; i++) {
        uint64_t cnt = 0, cells = (uint64_t)m->cfg.v_le * m->cfg.G;
        const uint16_t *row = m->LE + (uint64_t)i * cells;
        for (j = 0; j < cells; j++)
            if (row[j] < m->cfg.k) cnt++;
        m->row_fill[i] = cnt;
    }

    /* Eq8 */
    G = (double)m->cfg.G;
    v_le = (double)m->cfg.v_le;
    up = 1.0;
    for (i = 0; i < u; i++)
        up = up * ((double)m->row_fill[i] / (G * v_le));

    /* Eq9 for every candidate */
    for (x = 0; x < n; x++) {
        uint32_t aip = csip[x];
        uint32_t U = union_le_weight(m, aip);
        double num = (double)U - G * up;
        double den = G * (1.0 - up);
        double est;
        uint8_t fl = 0;
        if (den == 0.0) {
            est = INFINITY; fl |= ORC_SAT;
        } else {
            double xx = num / den;
            double y = 1.0 - xx;
            if (y <= 0.0) { est = INFINITY; fl |= ORC_SAT; }
            else est = -G * log(y);
        }
        if (est >= (double)m->cfg.theta) fl |= ORC_SUPER;
        if (x >= m->n_ncsip) fl |= ORC_NEW;
        m->r_est[x] = est;
        m->r_flags[x] = fl;
        m->r_U[x] = U;
        m->r_W[x] = (uint8_t)union_re_weight(m, aip);
    }

    /* Algorithm 3: clear every SI, slide every DR, keep the candidates whose
       union SRE still passes after the slide, and mark their SI bits */
    {
        uint64_t n_si = (uint64_t)u * m->cfg.v_re;
        uint64_t n_re = n_si * m->cfg.g;
        uint64_t n_le = (uint64_t)u * m->cfg.v_le * m->cfg.G;
        uint32_t *keep;
        uint64_t n_keep = 0;
        for (x = 0; x < n_si; x++) m->SI[x] = 0;
        for (x = 0; x < n_re; x++) DRslide(&m->RE[x]);
        for (x = 0; x < n_le; x++) DRslide(&m->LE[x]);
        m->slice++;
        keep = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
        if (!keep) { rc = -2; goto done; }
        for (x = 0; x < n; x++) {
            if (union_re_weight(m, csip[x]) >= m->t_re) {
                keep[n_keep++] = csip[x];
                m->r_flags[x] |= ORC_KEEP;
                set_si_bits(m, csip[x]);
            }
        }
        /* the carried list, ascending */
        if (n_keep) qsort(keep, n_keep, sizeof(uint32_t), cmp_u32);
        free(m->ncsip);
        m->ncsip = keep;
        m->n_ncsip = n_keep;
    }

    out->slice = m->slice - 1;
    out->window_full = (m->slice - 1) >= (uint64_t)(m->cfg.k - 1);
    out->n = n;
    out->ip = m->r_ip;
    out->est = m->r_est;
    out->flags = m->r_flags;
    out->union_weight = m->r_U;
    out->re_weight = m->r_W;
    out->row_fill = m->row_fill;
    out->up = up;
    out->n_touched = n_uniq;
    out->n_new = n_new;

done:
    m->n_touched = 0;
    m->n_seq_new = 0;
    free(uniq);
    free(news);
    return rc;
}

/* --------------------------------------------------------------- dumps */

/* Distances of every DR as of the open slice, with distances of 32768 and
   beyond written as 65535 (those DRs are outside every allowed window).
   which: 0 = LE, 1 = RE, 2 = SI (raw bits). */
int orc_dump(const orc_monitor *m, int which, uint16_t *out, uint64_t cells)
{
    uint64_t n, x;
    const uint16_t *src;
    if (!m || !out) return -1;
    if (which == 0) { n = (uint64_t)m->cfg.u * m->cfg.v_le * m->cfg.G; src = m->LE; }
    else if (which == 1) { n = (uint64_t)m->cfg.u * m->cfg.v_re * m->cfg.g; src = m->RE; }
    else if (which == 2) { n = (uint64_t)m->cfg.u * m->cfg.v_re; src = m->SI; }
    else return -1;
    if (cells != n) return -1;
    for (x = 0; x < n; x++) {
        uint16_t d = src[x];
        if (which != 2 && d >= 32768u) d = (uint16_t)DR_MAX;
        out[x] = d;
    }
    return 0;
}
