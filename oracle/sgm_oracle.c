/*
 * Plain CPU oracle for the semi-global-matching disparity path of
 * Ruf et al., "Real-time on-board obstacle avoidance for UAVs based on
 * embedded stereo vision" (arXiv 1807.06271).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may build, load or call
 * it; the GPU library never includes, links or calls anything here, and this
 * file uses nothing from the GPU library.
 *
 * Every step is integer arithmetic, written as plain nested loops over the
 * definitions, with int32/int64 intermediates and an explicit overflow check
 * where a value is stored in 16 bits.  No blocking, fusion or reordering
 * beyond what each definition states.  The optional OpenMP pragmas only split
 * independent scanlines / pixels across threads; results do not depend on the
 * thread count.
 *
 * Readings of the paper that this file fixes (each also listed with its
 * justification in the design notes of the repository):
 *  - Census bit = [I(q) < I(p)] (strict), neighbours visited in raster order
 *    (rows top to bottom, columns left to right, centre skipped), first
 *    neighbour in the most significant used bit; window coordinates are
 *    clamped to the image (edge replicate).
 *  - Cost of a disparity whose right pixel x - d falls left of the image is
 *    the Census bit count N_b (maximally dissimilar).
 *  - Aggregation is Hirschmueller's per-path recurrence: penalty 0 for the same
 *    disparity, P1 for a change of one, P2 otherwise, and after each pixel the
 *    minimum over disparities of the predecessor's path cost is subtracted.
 *    The first pixel of a path takes its matching cost unchanged.  The d-1
 *    term at d = 0 and the d+1 term at d = D-1 do not exist (no wrap).
 *  - WTA and the right-view disparity both take the smallest disparity on ties.
 *  - Left-right check: keep D_L(x,y) iff x - D_L >= 0 and
 *    |D_L - D_R(x - D_L, y)| <= lr_max_diff, else the invalid value.
 *  - Median of the k x k window with clamped coordinates, the invalid value
 *    taking part as its number.
 *  - U[d][x] counts rows y with D(x,y) = d; V[y][d] counts columns; values
 *    >= D (the invalid value) are not counted.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EOVERFLOW 1
#define ORACLE_EINVAL 2
#define ORACLE_ENOMEM 3

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Census transform (section 3.1.2, Census with Hamming distance after
 * Zabih and Woodfill 1994).  img has `pitch` bytes per row; out is [h][w]. */
int oracle_census(const uint8_t *img, int w, int h, int64_t pitch, int cw, int ch,
                  uint64_t *out) {
    if (w < 1 || h < 1 || cw < 1 || ch < 1 || !(cw & 1) || !(ch & 1) || cw * ch - 1 > 64)
        return ORACLE_EINVAL;
    int rx = (cw - 1) / 2, ry = (ch - 1) / 2;
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            uint8_t centre = img[(int64_t)y * pitch + x];
            uint64_t code = 0;
            for (int dy = -ry; dy <= ry; ++dy) {
                for (int dx = -rx; dx <= rx; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int qx = clampi(x + dx, 0, w - 1);
                    int qy = clampi(y + dy, 0, h - 1);
                    uint8_t v = img[(int64_t)qy * pitch + qx];
                    code = (code << 1) | (uint64_t)(v < centre ? 1 : 0);
                }
            }
            out[(int64_t)y * w + x] = code;
        }
    }
    return ORACLE_OK;
}

static int popcount64(uint64_t v) {
    int n = 0;
    while (v) { v &= v - 1; ++n; } /* clears the lowest set bit each time */
    return n;
}

/* Rectification by precomputed maps (section 3.1.1): for each pixel p of the
 * w x h rectified image, I_rect(p) = I(M_x(p), M_y(p)), where (M_x, M_y) are
 * integer source coordinates into the src_w x src_h raw image.  A map entry
 * outside the raw image gives 0 (no source pixel).  maps are [h][w]. */
int oracle_rectify(const uint8_t *src, int src_w, int src_h, int64_t src_pitch, const uint16_t *map_x,
                   const uint16_t *map_y, int w, int h, uint8_t *out) {
    if (src_w < 1 || src_h < 1 || w < 1 || h < 1) return ORACLE_EINVAL;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int sx = map_x[(int64_t)y * w + x], sy = map_y[(int64_t)y * w + x];
            out[(int64_t)y * w + x] = (sx < src_w && sy < src_h) ? src[(int64_t)sy * src_pitch + sx] : 0;
        }
    return ORACLE_OK;
}

/* Matching cost volume, equation (1): C(p, d) compares left pixel p with right
 * pixel (p_x - d, p_y) by the Hamming distance of their Census codes.
 * cost is [h][w][d_max]. */
int oracle_cost(const uint64_t *cl, const uint64_t *cr, int w, int h, int d_max, int nbits,
                uint16_t *cost) {
    if (w < 1 || h < 1 || d_max < 1) return ORACLE_EINVAL;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x)
            for (int d = 0; d < d_max; ++d) {
                int c;
                if (x - d >= 0)
                    c = popcount64(cl[(int64_t)y * w + x] ^ cr[(int64_t)y * w + (x - d)]);
                else
                    c = nbits;
                cost[((int64_t)y * w + x) * d_max + d] = (uint16_t)c;
            }
    return ORACLE_OK;
}

/* SAD matching cost (section 3.1.2, the sum of absolute differences over a
 * ww x wh support region, section 4.1): for 0 <= d < d_max,
 *   C(x,y,d) = sum over window offsets (dx,dy) of
 *              |I_L(x+dx, y+dy) - I_R(x-d+dx, y+dy)|
 * with every coordinate clamped to the image (each view on its own), and
 * C = ww*wh*255 (maximally dissimilar) where x - d < 0.  cost is
 * [h][w][d_max] uint16. */
int oracle_sad_cost(const uint8_t *left, const uint8_t *right, int w, int h, int64_t pitch, int ww,
                    int wh, int d_max, uint16_t *cost) {
    if (w < 1 || h < 1 || d_max < 1 || ww < 1 || wh < 1 || !(ww & 1) || !(wh & 1) || ww * wh * 255 > 65535)
        return ORACLE_EINVAL;
    int rx = ww / 2, ry = wh / 2;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x)
            for (int d = 0; d < d_max; ++d) {
                int c = 0;
                if (x - d < 0) {
                    c = ww * wh * 255;
                } else {
                    for (int dy = -ry; dy <= ry; ++dy)
                        for (int dx = -rx; dx <= rx; ++dx) {
                            int yy = clampi(y + dy, 0, h - 1);
                            int a = left[(int64_t)yy * pitch + clampi(x + dx, 0, w - 1)];
                            int b = right[(int64_t)yy * pitch + clampi(x - d + dx, 0, w - 1)];
                            c += a > b ? a - b : b - a;
                        }
                }
                cost[((int64_t)y * w + x) * d_max + d] = (uint16_t)c;
            }
    return ORACLE_OK;
}

/* Path directions r = (dx, dy), in the bit order of the path mask:
 * left-to-right, right-to-left, top-to-bottom, bottom-to-top, and the four
 * diagonals towards bottom-right, top-left, bottom-left, top-right. */
static const int DIR_DX[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
static const int DIR_DY[8] = {0, 0, +1, -1, +1, -1, +1, -1};

/* One pixel of one path (section 3.1.3, equation (2) read as Hirschmueller's
 * recurrence).  c: matching costs C(p, .); lp: the predecessor's path costs
 * L_r(p - r, .), or NULL at the start of the path; l: receives L_r(p, .).
 *   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d-1) + P1, L_r(p-r,d+1) + P1,
 *                           m + P2) - m,   m = min_k L_r(p-r,k). */
static void path_step(const uint16_t *c, const int32_t *lp, int32_t *l, int d_max, int p1, int p2) {
    if (!lp) {
        for (int d = 0; d < d_max; ++d) l[d] = c[d];
        return;
    }
    int32_t m = lp[0];
    for (int k = 1; k < d_max; ++k)
        if (lp[k] < m) m = lp[k];
    for (int d = 0; d < d_max; ++d) {
        int32_t best = lp[d];
        if (d >= 1 && lp[d - 1] + p1 < best) best = lp[d - 1] + p1;
        if (d + 1 < d_max && lp[d + 1] + p1 < best) best = lp[d + 1] + p1;
        if (m + p2 < best) best = m + p2;
        l[d] = (int32_t)c[d] + best - m;
    }
}

/* All scanlines of one path direction.  L is [h][w][d_max] int32 output.
 * Traversal: rows in the order of dy (any order when dy = 0), columns in the
 * order of dx (any order when dx = 0), so p - r is always done before p. */
static void path_cost(const uint16_t *cost, int w, int h, int d_max, int dir, int p1, int p2,
                      int32_t *L) {
    const int dx = DIR_DX[dir], dy = DIR_DY[dir];
#define ORACLE_PIXEL(x, y)                                                                   \
    do {                                                                                     \
        int px_ = (x) - dx, py_ = (y) - dy;                                                  \
        const int32_t *lp_ = (px_ < 0 || px_ >= w || py_ < 0 || py_ >= h)                   \
                                 ? NULL : L + ((int64_t)py_ * w + px_) * d_max;              \
        path_step(cost + ((int64_t)(y) * w + (x)) * d_max, lp_,                              \
                  L + ((int64_t)(y) * w + (x)) * d_max, d_max, p1, p2);                      \
    } while (0)
    if (dy == 0) {
        /* horizontal: rows are independent scanlines */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < h; ++y)
            for (int i = 0; i < w; ++i) ORACLE_PIXEL(dx > 0 ? i : w - 1 - i, y);
    } else {
        /* vertical / diagonal: each row only depends on the previous row */
        for (int j = 0; j < h; ++j) {
            int y = dy > 0 ? j : h - 1 - j;
#pragma omp parallel for schedule(static)
            for (int x = 0; x < w; ++x) ORACLE_PIXEL(x, y);
        }
    }
#undef ORACLE_PIXEL
}

/* Aggregated cost volume S(p, d) = sum over the paths in `mask` of L_r(p, d),
 * stored as uint16 [h][w][d_max].  Returns ORACLE_EOVERFLOW if any path cost
 * or sum exceeds 65535 (aggr then holds the low 16 bits).  With a single
 * bit in `mask`, aggr is that path's L_r. */
int oracle_aggregate(const uint16_t *cost, int w, int h, int d_max, uint32_t mask, int p1, int p2,
                     uint16_t *aggr) {
    if (w < 1 || h < 1 || d_max < 1 || mask == 0 || (mask & ~0xFFu) || p1 < 0 || p2 < 0)
        return ORACLE_EINVAL;
    int64_t n = (int64_t)w * h * d_max;
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *S = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!L || !S) { free(L); free(S); return ORACLE_ENOMEM; }
    int rc = ORACLE_OK;
    for (int dir = 0; dir < 8; ++dir) {
        if (!(mask & (1u << dir))) continue;
        path_cost(cost, w, h, d_max, dir, p1, p2, L);
        for (int64_t i = 0; i < n; ++i) {
            if (L[i] < 0 || L[i] > 65535) rc = ORACLE_EOVERFLOW;
            S[i] += L[i];
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (S[i] > 65535) rc = ORACLE_EOVERFLOW;
        aggr[i] = (uint16_t)S[i];
    }
    free(L);
    free(S);
    return rc;
}

/* Winner-takes-all (section 3.1.3): D_L(p) = argmin_d S(p, d), smallest d on
 * ties. */
void oracle_wta(const uint16_t *aggr, int w, int h, int d_max, uint16_t *disp) {
    for (int64_t p = 0; p < (int64_t)w * h; ++p) {
        const uint16_t *s = aggr + p * d_max;
        int best = 0;
        for (int d = 1; d < d_max; ++d)
            if (s[d] < s[best]) best = d;
        disp[p] = (uint16_t)best;
    }
}

/* Right-view disparity approximated from the left aggregated volume
 * (section 3.1.4): D_R(x, y) = argmin over d of S(x + d, y, d), for d with
 * x + d inside the image, smallest d on ties. */
void oracle_right_disparity(const uint16_t *aggr, int w, int h, int d_max, uint16_t *disp_r) {
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int best = 0;
            int32_t bestv = aggr[((int64_t)y * w + x) * d_max + 0];
            for (int d = 1; d < d_max && x + d < w; ++d) {
                int32_t v = aggr[((int64_t)y * w + x + d) * d_max + d];
                if (v < bestv) { bestv = v; best = d; }
            }
            disp_r[(int64_t)y * w + x] = (uint16_t)best;
        }
}

/* Left-right consistency check (section 3.1.4). */
void oracle_lr_check(const uint16_t *disp_l, const uint16_t *disp_r, int w, int h,
                     int max_diff, uint16_t invalid, uint16_t *out) {
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int dl = disp_l[(int64_t)y * w + x];
            int xr = x - dl;
            uint16_t v = invalid;
            if (xr >= 0) {
                int dr = disp_r[(int64_t)y * w + xr];
                int diff = dl - dr;
                if (diff < 0) diff = -diff;
                if (diff <= max_diff) v = (uint16_t)dl;
            }
            out[(int64_t)y * w + x] = v;
        }
}

static int cmp_u16(const void *a, const void *b) {
    return (int)*(const uint16_t *)a - (int)*(const uint16_t *)b;
}

/* k x k median filter (section 3.1.5), clamped borders; k odd, k <= 15. */
int oracle_median(const uint16_t *in, int w, int h, int k, uint16_t *out) {
    if (k < 1 || !(k & 1) || k > 15) return ORACLE_EINVAL;
    int r = k / 2;
    uint16_t win[225];
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int n = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx)
                    win[n++] = in[(int64_t)clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1)];
            qsort(win, (size_t)n, sizeof(uint16_t), cmp_u16);
            out[(int64_t)y * w + x] = win[n / 2];
        }
    return ORACLE_OK;
}

/* U-map and V-map (section 3.2): per-column and per-row histograms of the
 * disparity map.  umap is [d_max][w], vmap is [h][d_max]; values >= d_max
 * (the invalid marker) are not counted.  Returns ORACLE_EOVERFLOW if a count
 * exceeds 65535. */
int oracle_uv_maps(const uint16_t *disp, int w, int h, int d_max, uint16_t *umap, uint16_t *vmap) {
    int64_t nu = (int64_t)d_max * w, nv = (int64_t)h * d_max;
    uint32_t *u = (uint32_t *)calloc((size_t)nu, sizeof(uint32_t));
    uint32_t *v = (uint32_t *)calloc((size_t)nv, sizeof(uint32_t));
    if (!u || !v) { free(u); free(v); return ORACLE_ENOMEM; }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int d = disp[(int64_t)y * w + x];
            if (d >= d_max) continue;
            u[(int64_t)d * w + x] += 1;
            v[(int64_t)y * d_max + d] += 1;
        }
    int rc = ORACLE_OK;
    for (int64_t i = 0; i < nu; ++i) { if (u[i] > 65535) rc = ORACLE_EOVERFLOW; umap[i] = (uint16_t)u[i]; }
    for (int64_t i = 0; i < nv; ++i) { if (v[i] > 65535) rc = ORACLE_EOVERFLOW; vmap[i] = (uint16_t)v[i]; }
    free(u);
    free(v);
    return rc;
}

/* Obstacle-map filtering of a U- or V-map (section 3.2), in the paper's order:
 *  1. threshold:  b = 255 where count >= thr, else 0 (a binary map);
 *  2. dilation:   the maximum of b over the (2*dil_r+1)^2 square around each
 *                 cell, cells outside the map ignored;
 *  3. Gaussian:   the binomial kernel of size 2*blur_r+1 (weights
 *                 C(2*blur_r, blur_r+k), total 4^blur_r per axis) applied along
 *                 both axes with replicated borders, the 2-D sum rounded half up
 *                 after division by 4^(2*blur_r);
 *  4. region of interest: cells outside rows [roi_r0, roi_r1) and columns
 *                 [roi_c0, roi_c1) set to 0.
 * map: uint16 [rows][cols]; out: uint8 [rows][cols]. */
static int64_t binom(int n, int k) {
    int64_t c = 1;
    for (int i = 1; i <= k; ++i) c = c * (n - k + i) / i;
    return c;
}

int oracle_uv_filter(const uint16_t *map, int rows, int cols, int thr, int dil_r, int blur_r, int roi_r0,
                     int roi_r1, int roi_c0, int roi_c1, uint8_t *out) {
    if (rows < 1 || cols < 1 || dil_r < 0 || blur_r < 0 || blur_r > 4) return ORACLE_EINVAL;
    int64_t n = (int64_t)rows * cols;
    uint8_t *b = (uint8_t *)malloc((size_t)n), *dl = (uint8_t *)malloc((size_t)n);
    if (!b || !dl) { free(b); free(dl); return ORACLE_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) b[i] = map[i] >= thr ? 255 : 0;
    for (int y = 0; y < rows; ++y)
        for (int x = 0; x < cols; ++x) {
            uint8_t m = 0;
            for (int dy = -dil_r; dy <= dil_r; ++dy)
                for (int dx = -dil_r; dx <= dil_r; ++dx) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= rows || xx < 0 || xx >= cols) continue;
                    if (b[(int64_t)yy * cols + xx] > m) m = b[(int64_t)yy * cols + xx];
                }
            dl[(int64_t)y * cols + x] = m;
        }
    const int shift = 4 * blur_r;  /* log2 of 4^(2*blur_r) */
    for (int y = 0; y < rows; ++y)
        for (int x = 0; x < cols; ++x) {
            int64_t acc = 0;
            for (int i = -blur_r; i <= blur_r; ++i)
                for (int j = -blur_r; j <= blur_r; ++j) {
                    int yy = clampi(y + i, 0, rows - 1), xx = clampi(x + j, 0, cols - 1);
                    acc += binom(2 * blur_r, blur_r + i) * binom(2 * blur_r, blur_r + j) *
                           dl[(int64_t)yy * cols + xx];
                }
            int64_t g = shift ? (acc + ((int64_t)1 << (shift - 1))) >> shift : acc;
            int in_roi = y >= roi_r0 && y < roi_r1 && x >= roi_c0 && x < roi_c1;
            out[(int64_t)y * cols + x] = in_roi ? (uint8_t)g : 0;
        }
    free(b);
    free(dl);
    return ORACLE_OK;
}

/* Number of threads OpenMP would use (1 when built without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
