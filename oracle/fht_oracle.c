/*
 * CPU oracle for the dyadic-pattern fast Hough transform, plain C (C99 + OpenMP).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py load this library.  It shares no source, header,
 * table or helper with the HIP library in paper_2411_07351_amd/.
 *
 * It computes the transform by its definition (Sec. 3 of the paper): every line
 * summed by FHT2D is a vertical shift of a generating pattern built by Alg. 2,
 * so out[t][s] = sum_x A[x][(s + sigma * pat_{W,t}(x)) mod H].  No blocking,
 * fusion or reuse of partial sums: O(W^2 H) additions per quadrant, int64
 * accumulation for uint8 images and double accumulation for floating images.
 *
 * The rounding [.] of Alg. 2 is round-half-to-even on the exact rational
 * t (n_P - 1) / (n - 1); the quadrant views are q0 = V+ (lanes are image rows,
 * sign +1), q1 = V- (rows, -1), q2 = H+ (lanes are image columns, +1),
 * q3 = H- (columns, -1); positions wrap mod H.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define ORC_SPLIT_S 0
#define ORC_SPLIT_T 1

/* [.] of Alg. 2: nearest integer to num/den, ties to even (num >= 0, den > 0). */
static int64_t orc_rhe(int64_t num, int64_t den)
{
    int64_t q = num / den, r = num % den;
    if (2 * r > den) return q + 1;
    if (2 * r < den) return q;
    return q + (q & 1);
}

/* Split_S and Split_T of Sec. 3; returns the left width, the right is n - left. */
static int orc_split_left(int n, int split)
{
    if (split == ORC_SPLIT_S) return n / 2;
    int p = 1;                       /* largest power of two strictly below n */
    while (2 * p < n) p *= 2;
    return p;
}

/* Alg. 2: writes pat(n, t) + lift into out[0..n). */
static void orc_pattern_into(int n, int t, int split, int lift, int32_t *out)
{
    if (n == 1) { out[0] = lift; return; }
    int n0 = orc_split_left(n, split), n1 = n - n0;
    int t0 = (int)orc_rhe((int64_t)t * (n0 - 1), n - 1);
    int t1 = (int)orc_rhe((int64_t)t * (n1 - 1), n - 1);
    orc_pattern_into(n0, t0, split, lift, out);
    orc_pattern_into(n1, t1, split, lift + t - t1, out + n0);
}

int orc_patterns(int n, int split, int32_t *out)
{
    if (n < 1 || (split != ORC_SPLIT_S && split != ORC_SPLIT_T) || !out) return -1;
    for (int t = 0; t < n; ++t) orc_pattern_into(n, t, split, 0, out + (size_t)t * n);
    return 0;
}

int64_t orc_nonleaf_width_sum(int w, int split)
{
    if (w <= 1) return 0;
    int w0 = orc_split_left(w, split);
    return w + orc_nonleaf_width_sum(w0, split) + orc_nonleaf_width_sum(w - w0, split);
}

/* Lane-major copy A[x][y] of quadrant q, with W lanes and H positions. */
static void orc_view_dims(int q, int R, int C, int *W, int *H, int *sigma)
{
    *W = (q < 2) ? R : C;
    *H = (q < 2) ? C : R;
    *sigma = (q & 1) ? -1 : 1;
}

static int orc_bad_shape(int R, int C, int split)
{
    return R < 1 || C < 1 || (split != ORC_SPLIT_S && split != ORC_SPLIT_T);
}

/* uint8 image -> four int64 Hough images concatenated in q order. */
int orc_hough_u8(const uint8_t *img, int R, int C, int split, int64_t *out)
{
    if (!img || !out || orc_bad_shape(R, C, split)) return -1;
    size_t off = 0;
    for (int q = 0; q < 4; ++q) {
        int W, H, sigma;
        orc_view_dims(q, R, C, &W, &H, &sigma);
        uint8_t *A = (uint8_t *)malloc((size_t)W * H);
        int32_t *P = (int32_t *)malloc((size_t)W * W * sizeof(int32_t));
        if (!A || !P) { free(A); free(P); return -2; }
        for (int x = 0; x < W; ++x)
            for (int y = 0; y < H; ++y)
                A[(size_t)x * H + y] = (q < 2) ? img[(size_t)x * C + y] : img[(size_t)y * C + x];
        orc_patterns(W, split, P);
        int64_t *J = out + off;
        #pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < W; ++t) {
            int64_t *row = J + (size_t)t * H;
            for (int s = 0; s < H; ++s) row[s] = 0;
            for (int x = 0; x < W; ++x) {
                int64_t sh = ((int64_t)sigma * P[(size_t)t * W + x]) % H;
                if (sh < 0) sh += H;
                const uint8_t *lane = A + (size_t)x * H;
                int s = 0;
                for (; s < H - sh; ++s) row[s] += lane[s + sh];
                for (; s < H; ++s) row[s] += lane[s + sh - H];
            }
        }
        off += (size_t)W * H;
        free(A);
        free(P);
    }
    return 0;
}

/* double image -> four double Hough images and their per-line sums of |A|. */
int orc_hough_f64(const double *img, int R, int C, int split, double *out, double *absout)
{
    if (!img || !out || !absout || orc_bad_shape(R, C, split)) return -1;
    size_t off = 0;
    for (int q = 0; q < 4; ++q) {
        int W, H, sigma;
        orc_view_dims(q, R, C, &W, &H, &sigma);
        double *A = (double *)malloc((size_t)W * H * sizeof(double));
        int32_t *P = (int32_t *)malloc((size_t)W * W * sizeof(int32_t));
        if (!A || !P) { free(A); free(P); return -2; }
        for (int x = 0; x < W; ++x)
            for (int y = 0; y < H; ++y)
                A[(size_t)x * H + y] = (q < 2) ? img[(size_t)x * C + y] : img[(size_t)y * C + x];
        orc_patterns(W, split, P);
        double *J = out + off, *Ja = absout + off;
        #pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < W; ++t) {
            double *row = J + (size_t)t * H, *arow = Ja + (size_t)t * H;
            for (int s = 0; s < H; ++s) { row[s] = 0.0; arow[s] = 0.0; }
            for (int x = 0; x < W; ++x) {
                int64_t sh = ((int64_t)sigma * P[(size_t)t * W + x]) % H;
                if (sh < 0) sh += H;
                const double *lane = A + (size_t)x * H;
                for (int s = 0; s < H; ++s) {
                    double v = lane[(s + sh) % H];
                    row[s] += v;
                    arow[s] += v < 0 ? -v : v;
                }
            }
        }
        off += (size_t)W * H;
        free(A);
        free(P);
    }
    return 0;
}

/* Selected outputs (q[i], t[i], s[i]) of the uint8 transform, one by one. */
int orc_hough_sample_u8(const uint8_t *img, int R, int C, int split, int64_t n,
                        const int32_t *qs, const int32_t *ts, const int32_t *ss, int64_t *out)
{
    if (!img || !out || orc_bad_shape(R, C, split) || n < 0) return -1;
    int rc = 0;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int q = qs[i], W, H, sigma;
        if (q < 0 || q > 3) { rc = -1; continue; }
        orc_view_dims(q, R, C, &W, &H, &sigma);
        if (ts[i] < 0 || ts[i] >= W || ss[i] < 0 || ss[i] >= H) { rc = -1; continue; }
        int32_t *pat = (int32_t *)malloc((size_t)W * sizeof(int32_t));
        if (!pat) { rc = -2; continue; }
        orc_pattern_into(W, ts[i], split, 0, pat);
        int64_t acc = 0;
        for (int x = 0; x < W; ++x) {
            int64_t y = ((int64_t)ss[i] + (int64_t)sigma * pat[x]) % H;
            if (y < 0) y += H;
            acc += (q < 2) ? img[(size_t)x * C + y] : img[(size_t)y * C + x];
        }
        out[i] = acc;
        free(pat);
    }
    return rc;
}

/* Same for a double image; also the per-line sum of |A|. */
int orc_hough_sample_f64(const double *img, int R, int C, int split, int64_t n,
                         const int32_t *qs, const int32_t *ts, const int32_t *ss,
                         double *out, double *absout)
{
    if (!img || !out || !absout || orc_bad_shape(R, C, split) || n < 0) return -1;
    int rc = 0;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int q = qs[i], W, H, sigma;
        if (q < 0 || q > 3) { rc = -1; continue; }
        orc_view_dims(q, R, C, &W, &H, &sigma);
        if (ts[i] < 0 || ts[i] >= W || ss[i] < 0 || ss[i] >= H) { rc = -1; continue; }
        int32_t *pat = (int32_t *)malloc((size_t)W * sizeof(int32_t));
        if (!pat) { rc = -2; continue; }
        orc_pattern_into(W, ts[i], split, 0, pat);
        double acc = 0.0, aacc = 0.0;
        for (int x = 0; x < W; ++x) {
            int64_t y = ((int64_t)ss[i] + (int64_t)sigma * pat[x]) % H;
            if (y < 0) y += H;
            double v = (q < 2) ? img[(size_t)x * C + y] : img[(size_t)y * C + x];
            acc += v;
            aacc += v < 0 ? -v : v;
        }
        out[i] = acc;
        absout[i] = aacc;
        free(pat);
    }
    return rc;
}

/*
 * The whole pattern set P(w) (w x w, row t = pat(w, t)) by Alg. 2's recursion,
 * with the children's sets P(w0), P(w1) computed once and looked up instead of
 * being rebuilt per t.  A node's table is freed by the caller that made it.
 * Values are < w <= 32767, so int16 holds them.
 */
typedef struct { int w; int16_t *tab; } orc_memo;

static int16_t *orc_table(int w, int split, orc_memo *memo, int *nmemo)
{
    for (int i = 0; i < *nmemo; ++i)
        if (memo[i].w == w) return memo[i].tab;
    int16_t *tab = (int16_t *)malloc((size_t)w * w * sizeof(int16_t));
    if (!tab) return NULL;
    if (w == 1) {
        tab[0] = 0;
    } else {
        int w0 = orc_split_left(w, split), w1 = w - w0;
        int16_t *L = orc_table(w0, split, memo, nmemo);
        int16_t *R = orc_table(w1, split, memo, nmemo);
        if (!L || !R) { free(tab); return NULL; }
        for (int t = 0; t < w; ++t) {
            int t0 = (int)orc_rhe((int64_t)t * (w0 - 1), w - 1);
            int t1 = (int)orc_rhe((int64_t)t * (w1 - 1), w - 1);
            int16_t *row = tab + (size_t)t * w;
            memcpy(row, L + (size_t)t0 * w0, (size_t)w0 * sizeof(int16_t));
            for (int x = 0; x < w1; ++x) row[w0 + x] = (int16_t)(R[(size_t)t1 * w1 + x] + (t - t1));
        }
    }
    memo[*nmemo].w = w;
    memo[*nmemo].tab = tab;
    ++*nmemo;
    return tab;
}

/*
 * Sec. 4 / Sec. 5: for every n in [1, nmax], num[n] = max over t, x of
 * |x t - pat(n, t)(x) (n - 1)|, so that E(n) = num[n] / (n - 1) exactly
 * (num[1] = 0).  num has nmax + 1 entries; num[0] is set to 0.
 */
int orc_error_numerators(int nmax, int split, int64_t *num)
{
    if (nmax < 1 || nmax > 32767 || !num || (split != ORC_SPLIT_S && split != ORC_SPLIT_T))
        return -1;
    num[0] = 0;
    int rc = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int n = nmax; n >= 1; --n) {
        orc_memo memo[128];          /* a tree of width <= 32767 has < 128 distinct widths */
        int nmemo = 0;
        int16_t *P = orc_table(n, split, memo, &nmemo);
        if (!P) { rc = -2; }
        else {
            int64_t worst = 0;
            for (int t = 0; t < n; ++t) {
                const int16_t *row = P + (size_t)t * n;
                for (int x = 0; x < n; ++x) {
                    int64_t d = (int64_t)x * t - (int64_t)row[x] * (n - 1);
                    if (d < 0) d = -d;
                    if (d > worst) worst = d;
                }
            }
            num[n] = worst;
        }
        for (int i = 0; i < nmemo; ++i) free(memo[i].tab);
    }
    return rc;
}

/*
 * Alg. 1 itself, FHT2D(w, h, I, Split), for the uint8 -> int32 transform: the
 * paper's recursion, O(W H log W) additions per quadrant.  It is the CPU
 * counterpart of the GPU path for timing (the direct sums above are the
 * definition; tests check this recursion against them first).
 *
 * orc_alg1_rec computes the Hough image of lanes [a, a + w) of the lane-major
 * array A (W_all lanes of h positions) into rows [a, a + w) of dst, with tmp
 * as scratch of the same shape: both halves go to tmp (each using dst as its
 * own scratch), then row t of the result is row [t k0] of the left half plus
 * row [t k1] of the right half rotated by sigma (t - [t k1]) positions,
 * Rotate(v, r)[s] = v[(s + r) mod h].
 */
static void orc_alg1_rec(const uint8_t *A, int h, int a, int w, int split, int sigma,
                         int32_t *dst, int32_t *tmp)
{
    if (w == 1) {
        const uint8_t *lane = A + (size_t)a * h;
        int32_t *row = dst + (size_t)a * h;
        for (int s = 0; s < h; ++s) row[s] = lane[s];
        return;
    }
    int w0 = orc_split_left(w, split), w1 = w - w0;
    orc_alg1_rec(A, h, a, w0, split, sigma, tmp, dst);
    orc_alg1_rec(A, h, a + w0, w1, split, sigma, tmp, dst);
    for (int t = 0; t < w; ++t) {
        int t0 = (int)orc_rhe((int64_t)t * (w0 - 1), w - 1);
        int t1 = (int)orc_rhe((int64_t)t * (w1 - 1), w - 1);
        int64_t r = ((int64_t)sigma * (t - t1)) % h;
        if (r < 0) r += h;
        const int32_t *L = tmp + (size_t)(a + t0) * h;
        const int32_t *Rr = tmp + (size_t)(a + w0 + t1) * h;
        int32_t *row = dst + (size_t)(a + t) * h;
        int s = 0;
        for (; s < h - r; ++s) row[s] = L[s] + Rr[s + r];
        for (; s < h; ++s) row[s] = L[s] + Rr[s + r - h];
    }
}

/*
 * Alg. 1 over n images of R x C (row-major, back to back), all four
 * quadrants; outs receives each image's four int32 Hough images in q order
 * (4 R C int32 per image).  Images and quadrants are spread over the OpenMP
 * threads, each running the recursion on its own.  Returns 0, -1 on bad
 * arguments, -2 when out of memory.
 */
int orc_alg1_u8_batch(const uint8_t *imgs, int n, int R, int C, int split, int32_t *outs)
{
    if (!imgs || !outs || n < 0 || orc_bad_shape(R, C, split)) return -1;
    int rc = 0;
    const size_t px = (size_t)R * C;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t job = 0; job < (int64_t)n * 4; ++job) {
        const int i = (int)(job / 4), q = (int)(job % 4);
        int W, H, sigma;
        orc_view_dims(q, R, C, &W, &H, &sigma);
        const uint8_t *img = imgs + (size_t)i * px;
        uint8_t *A = (uint8_t *)malloc(px);
        int32_t *tmp = (int32_t *)malloc(px * sizeof(int32_t));
        if (!A || !tmp) { free(A); free(tmp); rc = -2; continue; }
        if (q < 2) {
            memcpy(A, img, px);
        } else {
            for (int x = 0; x < W; ++x)
                for (int y = 0; y < H; ++y) A[(size_t)x * H + y] = img[(size_t)y * C + x];
        }
        size_t off = (size_t)i * 4 * px + (q == 0 ? 0 : q == 1 ? px : q == 2 ? 2 * px : 3 * px);
        orc_alg1_rec(A, H, 0, W, split, sigma, outs + off, tmp);
        free(A);
        free(tmp);
    }
    return rc;
}

/* Threads an OpenMP parallel region of this library uses. */
int orc_num_threads(void)
{
    int n = 1;
    #pragma omp parallel
    {
        #pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
