/* Drives every oracle entry point on small random images (all shapes up to
 * 9 x 9, windows 1..19 and 255, gray and RGB) so that the CPU test suite can
 * run the oracle under AddressSanitizer and UBSan.  Exits 0 when every call
 * succeeds and its outputs are in range. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_binarize(const uint8_t *img, int H, int W, int channels, int win, double k, double R, int rule,
                    uint8_t *gray, uint32_t *s1, uint32_t *s2, uint32_t *n, double *m, double *s, double *t,
                    uint8_t *out);
int oracle_binarize_points(const uint8_t *img, int H, int W, int channels, int win, double k, double R,
                           int rule, const int32_t *ys, const int32_t *xs, int64_t npts, uint8_t *fval,
                           uint32_t *s1, uint32_t *s2, uint32_t *n, double *m, double *s, double *t,
                           uint8_t *out);
int oracle_otsu(const uint8_t *img, int H, int W, int channels, uint32_t *hist, int *kstar, uint8_t *out);
int oracle_binarize_gs(const uint8_t *img, int H, int W, int channels, int win, double k, double Rp,
                       int structure, uint32_t *s1, uint32_t *s2, uint32_t *n, double *t, uint8_t *out);

static uint64_t state = 88172645463325252ull;
static uint32_t next(void) {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)state;
}

int main(void) {
    const int wins[] = {1, 2, 3, 4, 5, 7, 9, 12, 15, 19, 255};
    int bad = 0, calls = 0;
    for (int H = 1; H <= 9; ++H)
        for (int W = 1; W <= 9; ++W)
            for (int C = 1; C <= 3; C += 2)
                for (size_t wi = 0; wi < sizeof wins / sizeof wins[0]; ++wi) {
                    const int win = wins[wi], npx = H * W;
                    uint8_t *img = malloc((size_t)npx * C), *gray = malloc(npx), *out = malloc(npx);
                    uint32_t *s1 = malloc(4 * npx), *s2 = malloc(4 * npx), *n = malloc(4 * npx);
                    double *m = malloc(8 * npx), *s = malloc(8 * npx), *t = malloc(8 * npx);
                    int32_t *ys = malloc(4 * npx), *xs = malloc(4 * npx);
                    for (int i = 0; i < npx * C; ++i) img[i] = (uint8_t)next();
                    for (int i = 0; i < npx; ++i) {
                        ys[i] = i / W;
                        xs[i] = i % W;
                    }
                    for (int rule = 0; rule <= 1; ++rule) {
                        const double k = rule == 0 ? 0.5 : -0.2;
                        bad |= oracle_binarize(img, H, W, C, win, k, 128.0, rule, gray, s1, s2, n, m, s, t, out) != 0;
                        bad |= oracle_binarize_points(img, H, W, C, win, k, 128.0, rule, ys, xs, npx, gray, s1, s2,
                                                      n, m, s, t, out) != 0;
                        for (int i = 0; i < npx; ++i) bad |= (out[i] != 0 && out[i] != 255) || n[i] < 1;
                        calls += 2;
                    }
                    uint32_t hist[256];
                    int kstar = -1;
                    bad |= oracle_otsu(img, H, W, C, hist, &kstar, out) < 0 || kstar < 0 || kstar > 255;
                    if (win % 2 == 1)
                        for (int st = 0; st < 3; ++st)
                            bad |= oracle_binarize_gs(img, H, W, C, win, 0.5, 128.0, st, s1, s2, n, t, out) != 0;
                    calls += 4;
                    free(img); free(gray); free(out); free(s1); free(s2); free(n);
                    free(m); free(s); free(t); free(ys); free(xs);
                }
    printf("%d oracle calls, %s\n", calls, bad ? "FAILED" : "ok");
    return bad;
}
