/*
 * Drives the oracle through its whole interface -- create, scan in pieces,
 * estimate, dump, sequential mode, capacity poisoning, invalid configs,
 * empty slices, k = 1 -- so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can check its memory accesses and arithmetic.
 * Exit status 0 on success; any sanitizer report aborts the run.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/srla_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint32_t next32(void)
{
    /* xorshift64* (Vigna 2016) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int run(orc_config cfg, int slices, uint64_t pairs_per_slice, uint32_t n_src)
{
    orc_monitor *m = orc_create(&cfg);
    uint32_t *pairs;
    uint16_t *dump;
    uint64_t cells = (uint64_t)cfg.u * cfg.v_le * cfg.G, x;
    int s, which, rc = 0;
    if (!m) return 1;
    pairs = (uint32_t *)malloc(2 * (pairs_per_slice + 1) * sizeof(uint32_t));
    dump = (uint16_t *)malloc(cells * sizeof(uint16_t));
    if (!pairs || !dump) return 2;
    for (s = 0; s < slices && rc == 0; s++) {
        orc_report r;
        uint64_t n = (s % 4 == 2) ? 0 : pairs_per_slice;   /* an empty slice now and then */
        for (x = 0; x < n; x++) {
            /* a heavy source, skewed ordinary sources, uniform destinations */
            uint32_t a = (x % 7 == 0) ? 7u : (next32() % n_src) * 2654435761u;
            pairs[2 * x] = a;
            pairs[2 * x + 1] = next32();
        }
        if (orc_scan(m, pairs, n / 2)) rc = 3;
        if (orc_scan(m, pairs + 2 * (n / 2), n - n / 2)) rc = 3;
        if (orc_estimate(m, &r) == 0) {
            double sum = 0.0;
            for (x = 0; x < r.n; x++) sum += r.flags[x] + (double)r.union_weight[x];
            if (sum < 0.0) rc = 4;
        }
        for (which = 0; which < 3 && rc == 0; which++) {
            uint64_t c = which == 0 ? cells
                       : which == 1 ? (uint64_t)cfg.u * cfg.v_re * cfg.g
                                    : (uint64_t)cfg.u * cfg.v_re;
            if (orc_dump(m, which, dump, c)) rc = 5;
        }
        if (orc_dump(m, 0, dump, cells + 1) == 0) rc = 6;   /* wrong size must fail */
    }
    orc_destroy(m);
    free(pairs);
    free(dump);
    return rc;
}

int main(void)
{
    orc_config c = {3, 64, 3, 64, 8, 8, 128, 11, 1u << 20, 0};
    orc_config bad = c;
    orc_report r;
    int rc;
    if ((rc = run(c, 9, 3000, 200))) return 10 + rc;
    c.sequential = 1;                                       /* Algorithm 2 in stream order */
    if ((rc = run(c, 7, 2000, 150))) return 20 + rc;
    c = (orc_config){1, 16, 16, 97, 64, 5, 4096, 12, 1u << 20, 0};   /* k = 1, u = 16, g = 64 */
    if ((rc = run(c, 5, 1500, 100))) return 30 + rc;
    c = (orc_config){4, 4, 4, 33, 3, 7, 192, 13, 1u << 20, 0};       /* tau = 0, odd sizes */
    if ((rc = run(c, 6, 1200, 300))) return 40 + rc;
    c = (orc_config){5, 64, 2, 64, 8, 8, 128, 14, 3, 0};             /* capacity 3: poisons */
    {
        orc_monitor *m = orc_create(&c);
        uint32_t p[2 * 400];
        int i, poisoned = 0;
        if (!m) return 50;
        for (i = 0; i < 400; i++) { p[2 * i] = (uint32_t)i % 40; p[2 * i + 1] = next32(); }
        for (i = 0; i < 4 && !poisoned; i++) {
            orc_scan(m, p, 400);
            poisoned = orc_estimate(m, &r) == -3;
        }
        if (!poisoned || orc_estimate(m, &r) != -4) return 51;
        orc_destroy(m);
    }
    bad.k = 0;
    if (orc_create(&bad)) return 60;
    bad = c; bad.G = 100;
    if (orc_create(&bad)) return 61;
    bad = c; bad.u = 17;
    if (orc_create(&bad)) return 62;
    if (orc_estimate(NULL, &r) != -1) return 63;
    orc_destroy(NULL);
    puts("ok");
    return 0;
}
