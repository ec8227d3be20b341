/* Vector-ALU throughput probe (measurement support, not part of the depth
   pipeline): the sustained rate of the integer instructions the SGM kernels
   are built from, so that a roofline's peak can be the smaller of the
   published figure and what the device does.  Library libvalu_peak.so. */
#ifndef VALU_PEAK_H
#define VALU_PEAK_H

#ifdef __cplusplus
extern "C" {
#endif

enum { kValuPeakOps = 8 };

/* Number of probed operations: 0 v_pk_add_u16, 1 v_pk_min_u16,
   2 v_pk_minimum3_f16, 3 v_add3_u32, 4 v_alignbit_b32, 5 v_bcnt_u32_b32,
   6 v_xor_b32, 7 v_min_u32 with a DPP row rotation. */
int valu_peak_ops(void);

/* Time `iters` loop trips (8 x 16 independent instructions each) of
   operation `op` on every lane of 8 blocks of 256 lanes per compute unit of
   the current device, on the null stream, after one warm-up launch.
   Writes wave instructions x 64 / seconds to *lane_ops_per_s (a packed
   instruction counts once) and the elapsed milliseconds to *ms.  Returns 0,
   1 for an invalid argument (op out of range, iters outside 1..2^20, null
   pointers), 2 for a HIP error.  Allocates and frees a small output buffer;
   synchronises the device. */
int valu_peak_measure(int op, int iters, double* lane_ops_per_s, double* ms);

#ifdef __cplusplus
}
#endif
#endif
