/* Floyd-Steinberg error diffusion of a probability map into a binary mask.
 * Used only to generate synthetic test and benchmark masks (the workload recipe
 * dithers a gradient-magnitude map); it is not part of the solver.
 * Raster order, threshold 0.5, weights 7/16 (right), 3/16 (below-left),
 * 5/16 (below), 1/16 (below-right). `p` is overwritten as scratch. */
#include <stdint.h>

void fs_dither(double *p, int64_t h, int64_t w, uint8_t *out)
{
    for (int64_t y = 0; y < h; ++y) {
        double *row = p + y * w;
        double *nxt = (y + 1 < h) ? p + (y + 1) * w : 0;
        for (int64_t x = 0; x < w; ++x) {
            double old = row[x];
            double q = old >= 0.5 ? 1.0 : 0.0;
            out[y * w + x] = (uint8_t)q;
            double e = old - q;
            if (x + 1 < w) row[x + 1] += e * (7.0 / 16.0);
            if (nxt) {
                if (x > 0) nxt[x - 1] += e * (3.0 / 16.0);
                nxt[x] += e * (5.0 / 16.0);
                if (x + 1 < w) nxt[x + 1] += e * (1.0 / 16.0);
            }
        }
    }
}
