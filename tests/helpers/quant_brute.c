/*
 * Exhaustive check of the oracle's BF16 and E4M3 encoders: every one of the
 * 2^32 FP32 bit patterns is encoded by the oracle and compared with a
 * brute-force search for the nearest value in the format's table of codes
 * (ties to the code with an even last fraction bit).  The table is built by
 * decoding every code, so the search shares nothing with the encoder.
 *   usage: quant_brute bf16|e4m3   -> prints the mismatch count
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_bf16_encode(const float*, int64_t, uint16_t*);
void oracle_e4m3_encode(const float*, int64_t, uint8_t*);
float oracle_e4m3_value(uint8_t);

static double tab_v[70000];
static uint32_t tab_c[70000];
static int ntab;

static int nearest_code(double a) {
    int lo = 0, hi = ntab - 1;
    if (a >= tab_v[hi]) return (int)tab_c[hi];
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (tab_v[mid] <= a) lo = mid; else hi = mid;
    }
    double dl = a - tab_v[lo], dh = tab_v[hi] - a;
    if (dl < dh) return (int)tab_c[lo];
    if (dh < dl) return (int)tab_c[hi];
    return (tab_c[lo] & 1) ? (int)tab_c[hi] : (int)tab_c[lo];
}

int main(int argc, char** argv) {
    int bf16 = argc > 1 && strcmp(argv[1], "bf16") == 0;
    if (bf16) {
        /* non-negative finite BF16 codes, then +inf standing at 2^128 (the
           value an unbounded exponent would round to) */
        for (uint32_t c = 0; c < 0x7F80; ++c) {
            uint32_t b = c << 16; float f; memcpy(&f, &b, 4);
            tab_v[ntab] = f; tab_c[ntab++] = c;
        }
        tab_v[ntab] = ldexp(1.0, 128); tab_c[ntab++] = 0x7F80;
    } else {
        for (uint32_t c = 0; c <= 0x7E; ++c) { tab_v[ntab] = oracle_e4m3_value((uint8_t)c); tab_c[ntab++] = c; }
    }
    long long bad = 0;
    const int64_t chunk = 1 << 20;
    #pragma omp parallel reduction(+ : bad)
    {
        float* x = malloc(sizeof(float) * chunk);
        uint16_t* h = malloc(sizeof(uint16_t) * chunk);
        uint8_t* q = malloc(chunk);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t base = 0; base < (1LL << 32); base += chunk) {
            for (int64_t i = 0; i < chunk; ++i) { uint32_t b = (uint32_t)(base + i); memcpy(&x[i], &b, 4); }
            if (bf16) oracle_bf16_encode(x, chunk, h); else oracle_e4m3_encode(x, chunk, q);
            for (int64_t i = 0; i < chunk; ++i) {
                uint32_t got = bf16 ? h[i] : q[i];
                uint32_t sign = signbit(x[i]) ? (bf16 ? 0x8000u : 0x80u) : 0u;
                uint32_t want;
                if (isnan(x[i])) {
                    /* NaN must stay NaN with its sign */
                    int ok = bf16 ? ((got & 0x7F80u) == 0x7F80u && (got & 0x7Fu) && (got & 0x8000u) == sign)
                                  : ((got & 0x7Fu) == 0x7Fu && (got & 0x80u) == sign);
                    bad += !ok;
                    continue;
                }
                double a = fabs((double)x[i]);
                if (!bf16 && a > 448.0) want = sign | 0x7Eu;      /* saturation */
                else want = sign | (uint32_t)nearest_code(a);
                bad += got != want;
            }
        }
        free(x); free(h); free(q);
    }
    printf("%lld\n", bad);
    return 0;
}
