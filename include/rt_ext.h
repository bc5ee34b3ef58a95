/*
 * rt_ext.h -- additional entry points of the gfx950 library, beside rt.h.
 * Same conventions as rt.h (device FP64 vectors of length N, hipStream_t as
 * void*, return codes, rt_last_error).
 */
#ifndef RT_EXT_H
#define RT_EXT_H

#include "rt.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * sigma_out = A sigma_in with the formal-solver sweep and quadrature of
 * Algorithm 1 carried out in FP32 (step coefficients rounded from their FP64
 * values, FP32 recurrences and accumulators; input read and output written in
 * FP64).  This is the operator of the inner solves of RT_PREC_MIXED; its error
 * against rt_apply_op is of the order of the FP32 unit roundoff times the
 * number of steps along a ray.  In-place allowed, as for rt_apply_op.
 */
int rt_apply_op_fp32(rt_handle *h, const double *sigma_in, double *sigma_out, void *stream);

/*
 * Describe the sweep plan: chunk length L, number of sweep workgroups, number
 * of stored coefficient pairs (tiles, including padding) and of ray-interval
 * pairs sum_slabs (ns - 1) (n_mu / 2) n_nu.  Any output pointer may be NULL.
 * Host only.
 */
int rt_plan_info(const rt_handle *h, int *chunk_L, int *n_blocks, long long *n_pairs,
                 long long *n_intervals);

/*
 * The sweep launch configuration of rt_apply_op (fp32 = 0) or
 * rt_apply_op_fp32 (fp32 != 0) on this handle: wavefronts per workgroup, and
 * 1 if the step coefficients of a wavefront's next ray batch are loaded while
 * the current one is swept, 0 if they are loaded on use.  Any output pointer
 * may be NULL.  Host only.
 */
int rt_sweep_config(const rt_handle *h, int fp32, int *waves, int *prefetch);

/*
 * Run the validation of rt_setup on (p, o) without touching any device:
 * RT_OK or RT_EINVAL with the message in rt_last_error().  o may be NULL.
 */
int rt_validate(const rt_problem *p, const rt_options *o);

#ifdef __cplusplus
}
#endif
#endif /* RT_EXT_H */
