/* Memory and undefined-behaviour check of the CPU oracle (test
 * infrastructure): built with gcc -fsanitize=address,undefined together with
 * oracle/oracle.c, it calls every oracle entry point on small seeded inputs
 * (grey and RGB, odd sizes, several bin counts and both orientations, hard
 * and soft votes, a pyramid, raw and L2 window scores) and checks a few
 * invariants that need no reference: the planes at the bottom-right corner
 * sum to the binned pixels, Eq. 5 equals its literal double sum, a cell holds
 * at most cell^2 pixels. Any sanitizer report aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_bin(int dx, int dy, int n_bins);
int orc_bin_table_ex(int n_bins, int unsigned_orientation, uint8_t *out);
int orc_bin_map_ex(const uint8_t *img, int w, int h, int channels, int64_t pitch, int n_bins,
                   int unsigned_orientation, uint8_t *out);
int orc_pyramid(int w, int h, double scale, int min_w, int min_h, int max_levels, int cap, int *lw,
                int *lh, double *ls);
int orc_resize_nn(const uint8_t *img, int w, int h, int channels, int64_t pitch, double s, int lw, int lh,
                  uint8_t *out);
int orc_integral(const uint8_t *bins, int w, int h, int n_bins, uint32_t *out);
int orc_integral_literal(const uint8_t *bins, int w, int h, int n_bins, uint32_t *out);
int orc_cell_hist(const uint8_t *bins, int w, int h, int n_bins, int cell, uint32_t *out);
int orc_soft_table(int n_bins, int unsigned_orientation, uint8_t *b0_out, uint8_t *w1_out);
int orc_soft_bin_map(const uint8_t *img, int w, int h, int channels, int64_t pitch, int n_bins,
                     int unsigned_orientation, uint8_t *b0_out, uint8_t *w1_out);
int orc_soft_integral(const uint8_t *b0, const uint8_t *w1, int w, int h, int n_bins, uint32_t *out);
int orc_soft_cell_hist(const uint8_t *b0, const uint8_t *w1, int w, int h, int n_bins, int cell,
                       uint32_t *out);
int orc_feature_dim(int n_bins, int wcx, int wcy, int block, int norm);
int orc_window_grid(int w, int h, int cell, int wcx, int wcy, int *nwx, int *nwy);
int orc_score_windows(const uint8_t *bins, int w, int h, int n_bins, int cell, int wcx, int wcy,
                      int block, int norm, double eps, const float *tmpl, const float *bias, int k_n,
                      int n_win, const int *wxs, const int *wys, double *scores, double *feats,
                      double *absterms);

static int failures = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

static uint32_t rng_state = 12345u;
static uint32_t rnd(void)
{
    rng_state = rng_state * 1664525u + 1013904223u;
    return rng_state >> 8;
}

static void one_image(int w, int h, int c, int nb, int orient)
{
    const int64_t pitch = (int64_t)w * c + 3; /* padded rows */
    uint8_t *img = malloc((size_t)pitch * h);
    for (int64_t i = 0; i < pitch * h; ++i) img[i] = (uint8_t)(rnd() & 255);
    uint8_t *bins = malloc((size_t)w * h);
    CHECK(orc_bin_map_ex(img, w, h, c, pitch, nb, orient, bins) == 0);
    int64_t binned = 0;
    for (int i = 0; i < w * h; ++i) binned += bins[i] != 255;
    uint32_t *ii = malloc((size_t)nb * (w + 1) * (h + 1) * sizeof(uint32_t));
    uint32_t *lit = malloc((size_t)nb * (w + 1) * (h + 1) * sizeof(uint32_t));
    CHECK(orc_integral(bins, w, h, nb, ii) == 0);
    int64_t corner = 0;
    for (int n = 0; n < nb; ++n) corner += ii[((int64_t)n * (h + 1) + h) * (w + 1) + w];
    CHECK(corner == binned);
    if (w * h <= 400) {
        CHECK(orc_integral_literal(bins, w, h, nb, lit) == 0);
        CHECK(memcmp(ii, lit, (size_t)nb * (w + 1) * (h + 1) * sizeof(uint32_t)) == 0);
    }
    const int cell = 8;
    if (w >= cell && h >= cell) {
        uint32_t *ch = malloc((size_t)(w / cell) * (h / cell) * nb * sizeof(uint32_t));
        CHECK(orc_cell_hist(bins, w, h, nb, cell, ch) == 0);
        for (int i = 0; i < (w / cell) * (h / cell); ++i) {
            uint32_t s = 0;
            for (int n = 0; n < nb; ++n) s += ch[(int64_t)i * nb + n];
            CHECK(s <= (uint32_t)(cell * cell));
        }
        free(ch);
    }
    /* Soft votes. */
    uint8_t *b0 = malloc((size_t)w * h), *w1 = malloc((size_t)w * h);
    CHECK(orc_soft_bin_map(img, w, h, c, pitch, nb, orient, b0, w1) == 0);
    CHECK(orc_soft_integral(b0, w1, w, h, nb, ii) == 0);
    if (w >= cell && h >= cell) {
        uint32_t *ch = malloc((size_t)(w / cell) * (h / cell) * nb * sizeof(uint32_t));
        CHECK(orc_soft_cell_hist(b0, w1, w, h, nb, cell, ch) == 0);
        free(ch);
    }
    /* Window scores, raw and L2, two templates. */
    for (int norm = 0; norm <= 1; ++norm) {
        const int wcx = 8, wcy = 16, block = 2;
        int nwx = 0, nwy = 0;
        CHECK(orc_window_grid(w, h, cell, wcx, wcy, &nwx, &nwy) == 0);
        if (nwx <= 0 || nwy <= 0) continue;
        const int dim = orc_feature_dim(nb, wcx, wcy, block, norm);
        CHECK(dim > 0);
        const int k = 2, n_win = nwx * nwy;
        float *t = malloc((size_t)k * dim * sizeof(float));
        float bias[2] = {0.5f, -1.f};
        for (int i = 0; i < k * dim; ++i) t[i] = (float)((int)(rnd() % 2001) - 1000) / 1000.f;
        int *wxs = malloc((size_t)n_win * sizeof(int)), *wys = malloc((size_t)n_win * sizeof(int));
        for (int i = 0; i < n_win; ++i) {
            wxs[i] = i % nwx;
            wys[i] = i / nwx;
        }
        double *sc = malloc((size_t)n_win * k * sizeof(double));
        double *ft = malloc((size_t)n_win * dim * sizeof(double));
        double *ab = malloc((size_t)n_win * k * sizeof(double));
        CHECK(orc_score_windows(bins, w, h, nb, cell, wcx, wcy, block, norm, 1e-3, t, bias, k, n_win,
                                wxs, wys, sc, ft, ab) == 0);
        for (int i = 0; i < n_win * k; ++i) CHECK(ab[i] >= 0.0);
        free(t);
        free(wxs);
        free(wys);
        free(sc);
        free(ft);
        free(ab);
    }
    /* Pyramid levels by nearest neighbour. */
    int lw[64], lh[64];
    double ls[64];
    const int nl = orc_pyramid(w, h, 1.1, 8, 8, 0, 64, lw, lh, ls);
    CHECK(nl >= 1);
    for (int l = 1; l < nl; ++l) {
        uint8_t *lv = malloc((size_t)lw[l] * lh[l] * c);
        CHECK(orc_resize_nn(img, w, h, c, pitch, ls[l], lw[l], lh[l], lv) == 0);
        uint8_t *lb = malloc((size_t)lw[l] * lh[l]);
        CHECK(orc_bin_map_ex(lv, lw[l], lh[l], c, (int64_t)lw[l] * c, nb, orient, lb) == 0);
        free(lb);
        free(lv);
    }
    free(b0);
    free(w1);
    free(lit);
    free(ii);
    free(bins);
    free(img);
}

int main(void)
{
    static uint8_t table[511 * 511], t0[511 * 511], t1[511 * 511];
    const int nbs[] = {1, 2, 8, 9, 18, 64};
    for (int i = 0; i < 6; ++i)
        for (int o = 0; o <= 1; ++o) {
            CHECK(orc_bin_table_ex(nbs[i], o, table) == 0);
            CHECK(orc_soft_table(nbs[i], o, t0, t1) == 0);
        }
    CHECK(orc_bin(0, 0, 8) == 255);
    const int sizes[][2] = {{1, 1}, {2, 3}, {7, 5}, {17, 13}, {64, 128}, {71, 133}, {90, 140}};
    for (int s = 0; s < 7; ++s)
        for (int c = 1; c <= 3; c += 2)
            for (int i = 0; i < 3; ++i) one_image(sizes[s][0], sizes[s][1], c, nbs[i * 2 + 1], (s + i) & 1);
    printf("%s\n", failures ? "FAIL" : "OK");
    return failures ? 1 : 0;
}
