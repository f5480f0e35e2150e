/*
 * cx_layout.h -- host-only introspection of what cx_create derives from a
 * station spec.  Neither call touches the GPU; they exist so that the spec
 * compiler and the sampling tables can be checked without a device.
 */
#ifndef CX_LAYOUT_H
#define CX_LAYOUT_H

#include "cx.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The capacity tree of Eq. (ArchConst) in the kernels' slot layout: every node
 * owns an aligned block of 2^b slots (children placed in port order, each
 * aligned to its own size), so each subtree sum is a butterfly over an aligned
 * lane group.  Outputs (host memory, caller-owned, may be NULL):
 *   *slots, *levels      padded slot count S (4..256) and tree depth D (1..4)
 *   slot_port [256]      port held by each slot, -1 for padding
 *   slot_lb   [256]      log2 of the block size per level (8 bits each, level 0 =
 *                        deepest), 0 where no node of that level covers the slot
 *   slot_cap  [4*256]    eta_H * I_H of the covering node per level ([level][slot]),
 *                        +inf where none
 * Returns CX_E_INVALID (with cx_last_error) for an invalid spec. */
cx_status cx_compile_layout(const cx_station_spec *spec, int32_t *slots, int32_t *levels,
                            int32_t *slot_port, uint32_t *slot_lb, float *slot_cap);

/* The integer sampling tables exactly as cx_create builds them (FP64 on the
 * host): tpois [steps_per_episode][24] arrival thresholds of Supp. B.1's Poisson
 * draw, tdwell [dwell_max] stay thresholds (entry 0 unused).  A word w gives
 * M = #{k : w > tpois[t][k]} arrivals and a stay of 1 + #{k >= 1 : w > tdwell[k]}. */
cx_status cx_build_tables(const cx_station_spec *spec, uint32_t *tpois, uint32_t *tdwell);

#ifdef __cplusplus
}
#endif
#endif
