/*
 * ash_ubench.h -- issue-rate microbenchmarks behind the transforms' issue
 * ceiling (libash_ubench.so, built beside libash.so).
 *
 * Every kernel evaluation of the transforms (one spot x one pixel) needs at
 * the least a hardware sine and cosine and an FP32 multiply-add per
 * accumulated component, and every 32 x 32 block of evaluations `groups`
 * 32x32x16 bf16 matrix-core products for its phases.  The ceiling on
 * evaluations per second is then
 *   simds * clock * 1024 / (32 trans + 32 fma + groups * mfma)
 * with the costs below, in cycles of the nominal clock per wave64
 * instruction per SIMD (vector and matrix-core issue measured separately;
 * on this chip they do not overlap).
 */
#ifndef ASH_UBENCH_H
#define ASH_UBENCH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ash_issue_rates {
  int simds;               /* 4 per compute unit                            */
  double nominal_clock_hz; /* 2.4e9                                         */
  double fma_cycles;       /* v_fma_f32, wave64, per SIMD                   */
  double trans_cycles;     /* v_sin_f32 / v_cos_f32 (alternating)           */
  double mfma_cycles;      /* v_mfma_f32_32x32x16_bf16                      */
  float ms[3];             /* shortest of three timed launches of each      */
} ash_issue_rates;

/* Time the three instruction streams on HIP device `device` with
 * waves_per_simd (1..8) resident waves on every SIMD (about 1 ms per
 * launch at 4).  Allocates and frees a small output buffer; synchronises
 * the device's null stream.  Returns 0,
 * -1 (bad argument), -5 (allocation failed) or -6 (HIP error). */
int ash_ubench_issue(int device, int waves_per_simd, ash_issue_rates* out);

/* Evaluations per second of the irreducible instruction mix of the
 * transforms' inner loop, without its loads, on every SIMD of `device` with
 * waves_per_simd (1..8) waves each: per 32 x 32 block of evaluations,
 * `groups` (1..12) dependent 32x32x16 bf16 matrix-core products for the
 * phases, then per phase (with reduce != 0 a range reduction) a sine and a
 * cosine, and two FMAs into per-lane sums (moments == 0: forward and
 * adjoint) or 8 further matrix-core products on the sines and cosines
 * (moments != 0: the moment transform).  This is the transforms' issue
 * ceiling on the chip (vector, transcendental and matrix-core issue overlap
 * partly, so the sum of the separate costs above overstates it).  Returns
 * 0, -1 (bad argument), -5 (allocation failed) or -6 (HIP error). */
int ash_ubench_mix(int device, int groups, int reduce, int moments,
                   int waves_per_simd, double* evals_per_s);

#ifdef __cplusplus
}
#endif

#endif /* ASH_UBENCH_H */
