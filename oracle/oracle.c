/*
 * oracle.c -- plain, slow, obviously correct CPU reference for exact locally
 * adaptive binarization (Mollah, Basu, Nasipuri, "Computationally Efficient
 * Implementation of Convolution-based Locally Adaptive Binarization
 * Techniques", arXiv:1210.3165).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * What it computes, per pixel (x, y), straight from the definitions:
 *   - gray level f (Sec. 1, Eq. 1): f = w_r r + w_g g + w_b b with the
 *     weights 0.299 / 0.587 / 0.114, evaluated exactly in integers as
 *     (299 r + 587 g + 114 b) / 1000 and rounded half up;
 *   - the W x W window S around the pixel (Sec. 2), clipped to the image;
 *     n = number of in-image window pixels;
 *   - S1 = sum of f over S, S2 = sum of f^2 over S (exact integers);
 *   - mean m = S1 / n and standard deviation s = sqrt(sum (f - m)^2 / n)
 *     (Sec. 1, the quantities of Eq. 4), taken as the population deviation,
 *     second pass over the window, in double precision;
 *   - threshold t (double): Sauvola, Eq. 4: t = m [1 + k (s / R - 1)];
 *     Niblack: t = m + k s;
 *   - binary output (Sec. 1, Eq. 3): g = 0 if f < t, 255 otherwise.
 *
 * And, for the paper's global baseline (Sec. 1, Eq. 2), Otsu's threshold:
 * the 256-bin histogram of f, the split level k* of largest between-class
 * variance and g = 0 if f < T = k* + 1 (oracle_otsu).
 *
 * And the sampled-window variant of Sec. 2 (Eq. 5) over this library's own
 * O(W) structures (oracle_binarize_gs).
 *
 * Window placement: rows [y - lo, y + hi], columns [x - lo, x + hi] with
 * lo = floor(win / 2), hi = win - 1 - lo, intersected with the image.
 *
 * Parity pins: every function here is checked by the CPU test suite against
 * brute force on tiny images, a summed-area table, closed forms and library
 * statistics; none of those checks reuses this code.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_RANGE (-2)
#define OR_ERR_NOMEM (-3)

int oracle_version(void) { return 1; }

/* Sec. 1, Eq. 1: gray level of one pixel. */
static uint8_t gray_pixel(const uint8_t *px, int channels) {
    if (channels == 1) return px[0];
    uint32_t num = 299u * px[0] + 587u * px[1] + 114u * px[2];
    /* round half up: floor(num / 1000 + 1/2) */
    return (uint8_t)((num + 500u) / 1000u);
}

/* Sec. 1, Eq. 1 over a whole image (H x W, interleaved channels). */
int oracle_gray(const uint8_t *img, int64_t H, int64_t W, int channels,
                uint8_t *gray) {
    if (!img || !gray || H < 0 || W < 0) return OR_ERR_ARG;
    if (channels != 1 && channels != 3) return OR_ERR_ARG;
    int64_t npx = H * W;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npx; ++i)
        gray[i] = gray_pixel(img + i * channels, channels);
    return OR_OK;
}

/* Everything the method determines for one pixel. */
typedef struct {
    uint32_t s1, s2, n;
    double m, s, t;
    uint8_t g;
} px_result;

/* Window statistics, threshold and decision for pixel (x, y) of the gray
 * image f (H x W).  rule 0 = Sauvola (Eq. 4), rule 1 = Niblack. */
static int pixel(const uint8_t *f, int H, int W, int win, double k, double R,
                 int rule, int y, int x, px_result *res) {
    int lo = win / 2, hi = win - 1 - lo;
    int ya = y - lo < 0 ? 0 : y - lo;
    int yb = y + hi > H - 1 ? H - 1 : y + hi;
    int xa = x - lo < 0 ? 0 : x - lo;
    int xb = x + hi > W - 1 ? W - 1 : x + hi;

    /* first pass over S: sums of f and f^2 */
    uint64_t a = 0, b = 0;
    for (int yy = ya; yy <= yb; ++yy)
        for (int xx = xa; xx <= xb; ++xx) {
            uint64_t v = f[(size_t)yy * W + xx];
            a += v;
            b += v * v;
        }
    uint64_t n = (uint64_t)(yb - ya + 1) * (uint64_t)(xb - xa + 1);
    if (a > 0xFFFFFFFFull || b > 0xFFFFFFFFull) return OR_ERR_RANGE;

    double m = (double)a / (double)n;

    /* second pass over S: population variance about the mean */
    double acc = 0.0;
    for (int yy = ya; yy <= yb; ++yy)
        for (int xx = xa; xx <= xb; ++xx) {
            double d = (double)f[(size_t)yy * W + xx] - m;
            acc += d * d;
        }
    double s = sqrt(acc / (double)n);

    double t;
    if (rule == 0)
        t = m * (1.0 + k * (s / R - 1.0)); /* Eq. 4 */
    else
        t = m + k * s; /* Niblack */

    res->s1 = (uint32_t)a;
    res->s2 = (uint32_t)b;
    res->n = (uint32_t)n;
    res->m = m;
    res->s = s;
    res->t = t;
    res->g = ((double)f[(size_t)y * W + x] < t) ? 0 : 255; /* Eq. 3 */
    return OR_OK;
}

static int check_args(const uint8_t *img, int H, int W, int channels, int win,
                      double R, int rule) {
    if (!img || H < 1 || W < 1) return OR_ERR_ARG;
    if (channels != 1 && channels != 3) return OR_ERR_ARG;
    if (win < 1 || win > 255) return OR_ERR_ARG;
    if (rule != 0 && rule != 1) return OR_ERR_ARG;
    if (rule == 0 && !(R > 0.0)) return OR_ERR_ARG;
    return OR_OK;
}

/*
 * Whole-image reference.  Every output pointer may be NULL except `out`.
 * gray: H*W u8; s1, s2, n: H*W u32; m, s, t: H*W f64; out: H*W u8.
 */
int oracle_binarize(const uint8_t *img, int H, int W, int channels, int win,
                    double k, double R, int rule, uint8_t *gray, uint32_t *s1,
                    uint32_t *s2, uint32_t *n, double *m, double *s, double *t,
                    uint8_t *out) {
    int rc = check_args(img, H, W, channels, win, R, rule);
    if (rc) return rc;
    if (!out) return OR_ERR_ARG;
    size_t npx = (size_t)H * (size_t)W;
    uint8_t *f = gray ? gray : (uint8_t *)malloc(npx);
    if (!f) return OR_ERR_NOMEM;
    oracle_gray(img, H, W, channels, f);

    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            px_result r;
            if (pixel(f, H, W, win, k, R, rule, y, x, &r)) {
                bad = 1;
                continue;
            }
            size_t i = (size_t)y * W + x;
            if (s1) s1[i] = r.s1;
            if (s2) s2[i] = r.s2;
            if (n) n[i] = r.n;
            if (m) m[i] = r.m;
            if (s) s[i] = r.s;
            if (t) t[i] = r.t;
            out[i] = r.g;
        }
    }
    if (!gray) free(f);
    return bad ? OR_ERR_RANGE : OR_OK;
}

/*
 * Sampled reference: the same quantities at npts chosen pixels (ys[i], xs[i])
 * of a large image, so that full-size launches can be checked point by point.
 * Every output array has npts entries; any may be NULL except out.
 */
int oracle_binarize_points(const uint8_t *img, int H, int W, int channels,
                           int win, double k, double R, int rule,
                           const int32_t *ys, const int32_t *xs, int64_t npts,
                           uint8_t *fval, uint32_t *s1, uint32_t *s2,
                           uint32_t *n, double *m, double *s, double *t,
                           uint8_t *out) {
    int rc = check_args(img, H, W, channels, win, R, rule);
    if (rc) return rc;
    if (!ys || !xs || !out || npts < 0) return OR_ERR_ARG;
    for (int64_t i = 0; i < npts; ++i)
        if (ys[i] < 0 || ys[i] >= H || xs[i] < 0 || xs[i] >= W) return OR_ERR_ARG;

    size_t npx = (size_t)H * (size_t)W;
    uint8_t *f = (uint8_t *)malloc(npx);
    if (!f) return OR_ERR_NOMEM;
    oracle_gray(img, H, W, channels, f);

    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t i = 0; i < npts; ++i) {
        px_result r;
        if (pixel(f, H, W, win, k, R, rule, ys[i], xs[i], &r)) {
            bad = 1;
            continue;
        }
        if (fval) fval[i] = f[(size_t)ys[i] * W + xs[i]];
        if (s1) s1[i] = r.s1;
        if (s2) s2[i] = r.s2;
        if (n) n[i] = r.n;
        if (m) m[i] = r.m;
        if (s) s[i] = r.s;
        if (t) t[i] = r.t;
        out[i] = r.g;
    }
    free(f);
    return bad ? OR_ERR_RANGE : OR_OK;
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int oracle_num_threads(void) {
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}

/*
 * Otsu's global threshold (the global baseline of Sec. 1, Eq. 2, whose
 * threshold the paper takes from Otsu's method).  From the 256-bin histogram
 * h of the gray levels (N pixels), for every level k the two classes are
 * C0 = {f <= k} and C1 = {f > k} with
 *   w0 = n0 / N, w1 = n1 / N, mu0 = S0 / n0, mu1 = S1 / n1
 * (n = pixel count, S = sum of levels of the class), and the between-class
 * variance is  sigma_b^2(k) = w0 w1 (mu0 - mu1)^2  (0 if a class is empty).
 * k* is the first level reaching the maximum; Eq. 2 then binarizes with
 * T = k* + 1 (g = 0 if f < T, i.e. f <= k*; 255 otherwise).
 * hist (256 u32), kstar and out may be NULL.  Returns T.
 */
static double otsu_sigma(uint64_t n0, uint64_t s0, uint64_t n, uint64_t s) {
    const uint64_t n1 = n - n0, s1 = s - s0;
    if (n0 == 0 || n1 == 0) return 0.0;
    const double w0 = (double)n0 / (double)n, w1 = (double)n1 / (double)n;
    const double mu0 = (double)s0 / (double)n0, mu1 = (double)s1 / (double)n1;
    const double d = mu0 - mu1;
    return w0 * w1 * (d * d);
}

int oracle_otsu(const uint8_t *img, int H, int W, int channels, uint32_t *hist, int *kstar,
                uint8_t *out) {
    if (!img || H < 1 || W < 1 || (channels != 1 && channels != 3)) return OR_ERR_ARG;
    size_t npx = (size_t)H * (size_t)W;
    uint8_t *f = (uint8_t *)malloc(npx);
    if (!f) return OR_ERR_NOMEM;
    oracle_gray(img, H, W, channels, f);
    uint64_t h[256] = {0};
    for (size_t i = 0; i < npx; ++i) h[f[i]]++;
    uint64_t n = npx, s = 0;
    for (int v = 0; v < 256; ++v) s += (uint64_t)v * h[v];
    int best = 0;
    double best_sigma = -1.0;
    uint64_t n0 = 0, s0 = 0;
    for (int k = 0; k < 256; ++k) {
        n0 += h[k];
        s0 += (uint64_t)k * h[k];
        const double sg = otsu_sigma(n0, s0, n, s);
        if (sg > best_sigma) {
            best_sigma = sg;
            best = k;
        }
    }
    const int T = best + 1;
    if (hist)
        for (int v = 0; v < 256; ++v) hist[v] = (uint32_t)h[v];
    if (kstar) *kstar = best;
    if (out)
        for (size_t i = 0; i < npx; ++i) out[i] = f[i] < T ? 0 : 255; /* Eq. 2 */
    free(f);
    return T;
}

/*
 * Sampled-window variant (Sec. 2, Eq. 5).  The paper replaces the window S by
 * a subset S' of O(W) pixels picked by a geometric structure (its Fig. 1,
 * whose drawings are not available).  The structures here are this
 * library's own, for odd win (lo = hi = win / 2), offsets (dy, dx) of the
 * window with
 *   structure 0 "plus":  dy == 0 or dx == 0          (centre row + column)
 *   structure 1 "x":     dy == dx or dy == -dx       (both diagonals)
 *   structure 2 "star":  the union of the two
 * clipped to the image; n' counts the in-image members.  m' = S1'/n',
 * s' = sqrt(sum (f - m')^2 / n') (second pass), t' = m' [1 + k (s'/R' - 1)]
 * (Eq. 5, R' the caller's dynamic range of s'), and g = 0 if f < t' (Eq. 3).
 * Every output pointer except out may be NULL.
 */
static int gs_member(int structure, int dy, int dx) {
    switch (structure) {
        case 0: return dy == 0 || dx == 0;
        case 1: return dy == dx || dy == -dx;
        case 2: return dy == 0 || dx == 0 || dy == dx || dy == -dx;
        default: return 0;
    }
}

int oracle_binarize_gs(const uint8_t *img, int H, int W, int channels, int win, double k,
                       double Rp, int structure, uint32_t *s1, uint32_t *s2, uint32_t *n,
                       double *t, uint8_t *out) {
    if (!img || !out || H < 1 || W < 1 || (channels != 1 && channels != 3)) return OR_ERR_ARG;
    if (win < 1 || win > 255 || win % 2 == 0) return OR_ERR_ARG;
    if (structure < 0 || structure > 2 || !(Rp > 0.0)) return OR_ERR_ARG;
    const int r = win / 2;
    /* the members of S' as offsets from the centre */
    int *dys = (int *)malloc(sizeof(int) * (size_t)win * win);
    int *dxs = (int *)malloc(sizeof(int) * (size_t)win * win);
    size_t npx = (size_t)H * (size_t)W;
    uint8_t *f = (uint8_t *)malloc(npx);
    if (!dys || !dxs || !f) {
        free(dys);
        free(dxs);
        free(f);
        return OR_ERR_NOMEM;
    }
    int nm = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            if (gs_member(structure, dy, dx)) {
                dys[nm] = dy;
                dxs[nm] = dx;
                ++nm;
            }
    oracle_gray(img, H, W, channels, f);
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            uint64_t a = 0, b = 0, cnt = 0;
            for (int i = 0; i < nm; ++i) {
                const int yy = y + dys[i], xx = x + dxs[i];
                if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                const uint64_t v = f[(size_t)yy * W + xx];
                a += v;
                b += v * v;
                ++cnt;
            }
            const double m = (double)a / (double)cnt;
            double acc = 0.0;
            for (int i = 0; i < nm; ++i) {
                const int yy = y + dys[i], xx = x + dxs[i];
                if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                const double d = (double)f[(size_t)yy * W + xx] - m;
                acc += d * d;
            }
            const double s = sqrt(acc / (double)cnt);
            const double tt = m * (1.0 + k * (s / Rp - 1.0)); /* Eq. 5 */
            const size_t i = (size_t)y * W + x;
            if (s1) s1[i] = (uint32_t)a;
            if (s2) s2[i] = (uint32_t)b;
            if (n) n[i] = (uint32_t)cnt;
            if (t) t[i] = tt;
            out[i] = ((double)f[i] < tt) ? 0 : 255; /* Eq. 3 */
        }
    free(dys);
    free(dxs);
    free(f);
    return OR_OK;
}
