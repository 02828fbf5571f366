/*
 * synth_cpu.c — seeded synthetic inputs, CPU build (plain C + OpenMP).
 *
 * Input generator only: random simulation parameters, the per-voxel
 * concentration volumes (via synth_formula.h, shared with the GPU build) and
 * the noisy patient-segmentation stand-ins used as queries. The retrieval
 * method itself (thresholds applied to the database, overlaps, Dice, ranking)
 * lives elsewhere; this file only manufactures the data the paper's database
 * (Sec. 3 "Data") and patient scans would have provided.
 *
 * Random numbers come from one counter-based generator: SplitMix64 chained
 * over (seed, item, draw):
 *     h = mix(mix(mix(seed) ^ item) ^ draw),  u = (h >> 11) * 2^-53  in [0, 1)
 * where mix is Vigna's SplitMix64 output function (add the golden-ratio
 * increment, then two xor-shift-multiply rounds and a final xor-shift).
 * Every value therefore depends only on its (seed, item, draw) triple and
 * not on thread count or call order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "synth_formula.h"

static uint64_t sm64_mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_hash(uint64_t seed, int64_t item, uint64_t draw)
{
    return sm64_mix(sm64_mix(sm64_mix(seed) ^ (uint64_t)item) ^ draw);
}

double synth_uniform(uint64_t seed, int64_t item, uint64_t draw)
{
    return (double)(synth_hash(seed, item, draw) >> 11) * (1.0 / 9007199254740992.0);
}

/* Brain mask of a grid: centre (n-1)/2, semi-axes (0.40, 0.46, 0.36) * n. */
void synth_brain(int nx, int ny, int nz, synth_brain_t *b)
{
    b->Cx = (nx - 1) * 0.5;
    b->Cy = (ny - 1) * 0.5;
    b->Cz = (nz - 1) * 0.5;
    b->iAx = 1.0 / (0.40 * nx);
    b->iAy = 1.0 / (0.46 * ny);
    b->iAz = 1.0 / (0.36 * nz);
}

/*
 * Parameters of simulations n0 .. n0+count-1.
 * Draws 0..191: up to 64 rejection attempts for a centre uniform in the brain
 * ellipsoid (u in [-1,1]^3 accepted when |u| <= 1; centre = C + A*u).
 * Draws 200..204: R ~ U[r_lo, r_hi], w ~ U[w_lo, w_hi], a_d ~ U[0.7, 1.3].
 */
void synth_params(uint64_t seed, int64_t n0, int64_t count, int nx, int ny, int nz,
                  double r_lo, double r_hi, double w_lo, double w_hi, synth_params_t *out)
{
    double Ax = 0.40 * nx, Ay = 0.46 * ny, Az = 0.36 * nz;
    double Cx = (nx - 1) * 0.5, Cy = (ny - 1) * 0.5, Cz = (nz - 1) * 0.5;
    for (int64_t t = 0; t < count; ++t) {
        int64_t n = n0 + t;
        double ux = 0.0, uy = 0.0, uz = 0.0;
        for (int a = 0; a < 64; ++a) {
            double vx = 2.0 * synth_uniform(seed, n, 3 * a + 0) - 1.0;
            double vy = 2.0 * synth_uniform(seed, n, 3 * a + 1) - 1.0;
            double vz = 2.0 * synth_uniform(seed, n, 3 * a + 2) - 1.0;
            if (vx * vx + vy * vy + vz * vz <= 1.0) {
                ux = vx;
                uy = vy;
                uz = vz;
                break;
            }
        }
        synth_params_t *p = &out[t];
        p->cx = Cx + Ax * ux;
        p->cy = Cy + Ay * uy;
        p->cz = Cz + Az * uz;
        p->R = r_lo + (r_hi - r_lo) * synth_uniform(seed, n, 200);
        double w = w_lo + (w_hi - w_lo) * synth_uniform(seed, n, 201);
        p->iw = 1.0 / w;
        p->iax = 1.0 / (0.7 + 0.6 * synth_uniform(seed, n, 202));
        p->iay = 1.0 / (0.7 + 0.6 * synth_uniform(seed, n, 203));
        p->iaz = 1.0 / (0.7 + 0.6 * synth_uniform(seed, n, 204));
    }
}

/* Concentration volumes [count][nz][ny][nx] float32, x fastest. */
void synth_fill_cpu(const synth_params_t *p, int64_t count, int nx, int ny, int nz, float *out,
                    int nthreads)
{
    synth_brain_t b;
    synth_brain(nx, ny, nz, &b);
    int64_t planes = count * (int64_t)nz;
    int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t s = 0; s < planes; ++s) {
        int64_t t = s / nz;
        int k = (int)(s % nz);
        float *o = out + t * (int64_t)nz * plane + (int64_t)k * plane;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                o[(int64_t)j * nx + i] = synth_conc(&p[t], &b, i, j, k);
    }
}

/* Voxels of one mask bit that have an in-grid 6-neighbour with the other value. */
static int64_t boundary_list(const uint8_t *lab, int bit, int nx, int ny, int nz, int64_t *list)
{
    int64_t nb = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t v = ((int64_t)k * ny + j) * nx + i;
                int val = (lab[v] >> bit) & 1;
                int diff = 0;
                if (i > 0 && ((lab[v - 1] >> bit) & 1) != val) diff = 1;
                if (i + 1 < nx && ((lab[v + 1] >> bit) & 1) != val) diff = 1;
                if (j > 0 && ((lab[v - nx] >> bit) & 1) != val) diff = 1;
                if (j + 1 < ny && ((lab[v + nx] >> bit) & 1) != val) diff = 1;
                if (k > 0 && ((lab[v - (int64_t)nx * ny] >> bit) & 1) != val) diff = 1;
                if (k + 1 < nz && ((lab[v + (int64_t)nx * ny] >> bit) & 1) != val) diff = 1;
                if (diff)
                    list[nb++] = v;
            }
    return nb;
}

/*
 * A synthetic patient segmentation: simulation p segmented at (t_lo, t_hi)
 * into bit 0 (FLAIR, c >= t_lo) and bit 1 (T1Gd, c >= t_hi), then, per mask
 * independently, round(flip_frac * |boundary|) boundary voxels flipped,
 * chosen by a partial Fisher-Yates shuffle driven by (noise_seed, qid).
 * Both boundary sets are taken before any flip. nflip[2] receives the flip
 * counts. Returns 0, or -1 if scratch memory could not be allocated.
 */
int synth_query_labels(const synth_params_t *p, int nx, int ny, int nz, float t_lo, float t_hi,
                       uint64_t noise_seed, int64_t qid, double flip_frac, uint8_t *labels,
                       int64_t *nflip)
{
    synth_brain_t b;
    synth_brain(nx, ny, nz, &b);
    int64_t V = (int64_t)nx * ny * nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                float c = synth_conc(p, &b, i, j, k);
                labels[((int64_t)k * ny + j) * nx + i] =
                    (uint8_t)((c >= t_lo ? 1 : 0) | (c >= t_hi ? 2 : 0));
            }
    int64_t *lists[2];
    int64_t counts[2];
    lists[0] = (int64_t *)malloc(sizeof(int64_t) * (size_t)V);
    lists[1] = (int64_t *)malloc(sizeof(int64_t) * (size_t)V);
    if (!lists[0] || !lists[1]) {
        free(lists[0]);
        free(lists[1]);
        return -1;
    }
    for (int m = 0; m < 2; ++m)
        counts[m] = boundary_list(labels, m, nx, ny, nz, lists[m]);
    for (int m = 0; m < 2; ++m) {
        int64_t nb = counts[m];
        int64_t kf = (int64_t)floor(flip_frac * (double)nb + 0.5);
        if (kf > nb) kf = nb;
        int64_t *L = lists[m];
        for (int64_t i = 0; i < kf; ++i) {
            double u = synth_uniform(noise_seed, qid, ((uint64_t)m << 40) | (uint64_t)i);
            int64_t j = i + (int64_t)floor(u * (double)(nb - i));
            if (j >= nb) j = nb - 1;
            int64_t tmp = L[i];
            L[i] = L[j];
            L[j] = tmp;
            labels[L[i]] ^= (uint8_t)(1u << m);
        }
        if (nflip) nflip[m] = kf;
    }
    free(lists[0]);
    free(lists[1]);
    return 0;
}
