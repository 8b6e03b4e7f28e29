/*
 * pf_debug.h - self-checks of the symbolic analysis and of the
 * preconditioner set-up.
 *
 * Not a compute path: the solve entry points of pf.h never call these.  The
 * two analysis checks touch no device, so that the fill-reducing ordering and
 * the symbolic block LU of Sec. III-A can be tested on a machine without a
 * GPU; the preconditioner check runs its set-up kernels on the device.
 */
#ifndef PF_DEBUG_H_
#define PF_DEBUG_H_

#include <stdint.h>

#include "pf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Analyse the case described by `desc` exactly as pf_create_scheduled does
 * under `sched` (NULL: the default schedule; same validation, PF_E_INVALID on
 * bad input), then replay on the CPU every index
 * the device kernels derive from that analysis: the Ybus-to-factor map, the
 * update lists of each refactorisation level, the Schur lists of the dense
 * block and the row lists of both triangular solves.  Every index is
 * bounds-checked and every dependency checked against the level schedule
 * (a failed check returns PF_E_INVALID with the reason in pf_last_error()).
 * A random diagonally dominant 2x2-block matrix with the Ybus pattern (seeded
 * by `seed`) is factored through the schedule and one random system solved;
 * *rel_residual receives ||A x - b||_inf / (||A||_inf ||x||_inf + ||b||_inf)
 * and *checks the number of index checks made.  Outputs are host pointers. */
pf_status pf_debug_schedule_check(const pf_case_desc* desc, const pf_schedule* sched, uint64_t seed,
                                  double* rel_residual, int64_t* checks);

/* The same for the Newton-Krylov inner solve (Sec. III-B): analyse the case
 * as pf_create does, check every index of the Krylov analysis (ordering,
 * 2x2-block pattern, Ybus-to-block map, ILU(0) update lists, the forward and
 * backward level schedules, block-Jacobi groups), then factor a random
 * diagonally dominant matrix on that pattern with block ILU(0) through the
 * update lists in level order and apply it through both schedules.
 * *ilu_deviation receives max |(L U - A)_ij| / max |A_ij| over the pattern
 * (ILU(0) reproduces A there), *rel_residual the relative residual of
 * L U z = v, *checks the number of checks.  PF_E_INVALID on a failed check
 * (reason in pf_last_error()).  Outputs are host pointers. */
pf_status pf_debug_krylov_check(const pf_case_desc* desc, uint64_t seed, double* ilu_deviation,
                                double* rel_residual, int64_t* checks);

/* The one call here that uses the device: a check of the Newton-Krylov
 * preconditioner set-up kernels (Sec. III-B).  The case's Jacobian at its
 * flat start is built on the device and the set-up kernels for `precond`
 * run on it exactly as in a Krylov Newton step (FP64); the results are
 * copied back and checked on the host against their definitions:
 *   PF_PRECOND_ILU0:    *deviation = max over the pattern of
 *                       |(L U - A)_ij| / max |A_ij|, together with
 *                       max |U_rr Uinv_rr - I| of the stored inverted
 *                       diagonal blocks; *max_order = 2 (block order);
 *   PF_PRECOND_BJACOBI: *deviation = max over the node groups of
 *                       max |A_bb X - I|, X the stored inverse of the group's
 *                       diagonal block A_bb; *max_order = the largest group
 *                       order (2 x nodes).
 * The case is left at its flat-start voltage.  Host outputs.  PF_E_BUSY while
 * the case is queued or running; PF_E_INVALID for a singular pivot. */
pf_status pf_debug_precond_check(pf_case* c, int32_t precond, double* deviation, int32_t* max_order);

#ifdef __cplusplus
}
#endif

#endif /* PF_DEBUG_H_ */
