/*
 * synth_formula.h — per-voxel value of one synthetic tumour volume.
 *
 * Seeded input generator, shared by the CPU build (synth_cpu.c, gcc) and the
 * GPU build (synth_gpu.hip, hipcc) of the same definition, so that both write
 * identical float32 bytes for a simulation. It holds none of the retrieval
 * method's arithmetic (no thresholds, no overlaps, no ranking): it only makes
 * the stand-in for the paper's pre-simulated tumour density u in [0,1]
 * (Sec. 2.1, "Tumor growth model"; Sec. 3 "Data" describes the 50k database
 * on a 128^3 grid, which is not available and is replaced by this generator).
 *
 * The stand-in is a logistic front around a random centre inside an
 * ellipsoidal brain mask:
 *     c(p) = brain(p) ? 1 / (1 + exp((r_aniso(p) - R) / w)) : 0
 *     r_aniso(p) = sqrt(sum_d ((p_d - c_d) * inv_a_d)^2)
 * evaluated in double and rounded once to float32.
 *
 * Bit-identical CPU/GPU results rest on using only correctly rounded IEEE
 * double operations (+, -, *, /, sqrt, floor, ldexp) in one fixed order with
 * no fused multiply-add contraction (both builds pass -ffp-contract=off and
 * clang additionally sees the pragma below). exp() is NOT taken from either
 * math library: synth_exp() is Cody-Waite range reduction by ln 2 followed by
 * the degree-13 Taylor polynomial of e^r on |r| <= ln2/2, evaluated by Horner.
 * Its truncation error, (ln2/2)^14/14! ~ 4e-18, is below half an ulp of 1.
 *
 * Two clamps are part of the definition: x = (r - R)/w > 80 gives c = 0
 * (the logistic is then below the smallest normal float, so no float32
 * denormals are ever written) and x < -40 gives c = 1 (1/(1+e^-40) already
 * rounds to 1.0 in double).
 */
#ifndef SYNTH_FORMULA_H
#define SYNTH_FORMULA_H

#if defined(__HIPCC__)
#define SYNTH_FN __host__ __device__ static inline
#else
#include <math.h>
#define SYNTH_FN static inline
#endif

/* Per-simulation parameters, computed once on the host from the seed. */
typedef struct {
    double cx, cy, cz;     /* front centre, voxel units (x fastest) */
    double iax, iay, iaz;  /* reciprocal anisotropy 1/a_d */
    double R;              /* front radius, voxels */
    double iw;             /* reciprocal front width 1/w */
} synth_params_t;

/* The ellipsoidal brain mask, shared by all simulations of a grid. */
typedef struct {
    double Cx, Cy, Cz;     /* centre ((n_d - 1) / 2) */
    double iAx, iAy, iAz;  /* reciprocal semi-axes */
} synth_brain_t;

SYNTH_FN double synth_exp(double x)
{
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    const double inv_ln2 = 1.4426950408889634;
    const double ln2_hi = 6.93147180369123816490e-01; /* low 32 bits zero */
    const double ln2_lo = 1.90821492927058770002e-10;
    double kd = floor(x * inv_ln2 + 0.5);
    double r = (x - kd * ln2_hi) - kd * ln2_lo;
    /* 1/n! for n = 13 .. 2, each the correctly rounded double. */
    double p = 1.6059043836821613e-10;
    p = p * r + 2.08767569878681e-09;
    p = p * r + 2.505210838544172e-08;
    p = p * r + 2.755731922398589e-07;
    p = p * r + 2.7557319223985893e-06;
    p = p * r + 2.48015873015873e-05;
    p = p * r + 0.0001984126984126984;
    p = p * r + 0.001388888888888889;
    p = p * r + 0.008333333333333333;
    p = p * r + 0.041666666666666664;
    p = p * r + 0.16666666666666666;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)kd);
}

SYNTH_FN int synth_in_brain(const synth_brain_t *b, int i, int j, int k)
{
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    double ux = ((double)i - b->Cx) * b->iAx;
    double uy = ((double)j - b->Cy) * b->iAy;
    double uz = ((double)k - b->Cz) * b->iAz;
    return ((ux * ux + uy * uy) + uz * uz) <= 1.0;
}

/* Concentration at voxel (i, j, k) = (x, y, z). */
SYNTH_FN float synth_conc(const synth_params_t *p, const synth_brain_t *b, int i, int j, int k)
{
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    if (!synth_in_brain(b, i, j, k))
        return 0.0f;
    double dx = ((double)i - p->cx) * p->iax;
    double dy = ((double)j - p->cy) * p->iay;
    double dz = ((double)k - p->cz) * p->iaz;
    double r = sqrt((dx * dx + dy * dy) + dz * dz);
    double x = (r - p->R) * p->iw;
    if (x > 80.0)
        return 0.0f;
    if (x < -40.0)
        return 1.0f;
    return (float)(1.0 / (1.0 + synth_exp(x)));
}

#endif /* SYNTH_FORMULA_H */
