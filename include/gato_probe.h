/*
 * gato_probe.h - measurement aid of the MI355X trajectory-optimisation library
 * (not part of the solver): the LDS read bandwidth of the device, the peak
 * against which the solver kernels' LDS traffic is reported beside their
 * arithmetic rate.
 */
#ifndef GATO_PROBE_H
#define GATO_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Runs one 512-thread workgroup per CU on the current device, each reading
 * 16-byte vectors from its LDS `iters` x 16 times (a warm-up launch, then a
 * timed one on the null stream; synchronous). pattern 0: every lane reads its
 * own 16 bytes (consecutive lanes, consecutive addresses); pattern 1: each
 * group of 16 lanes reads the same 16 bytes (broadcast). Outputs (host
 * pointers, may be NULL): delivered bytes (16 per lane per load) per shader
 * clock per CU, from the slowest workgroup's clock counter; and delivered
 * bytes per second over the whole device, from HIP events. Allocates and frees
 * small device buffers. Returns 0, -1 for bad arguments (pattern not 0/1,
 * iters outside 1..2^20), -2 on allocation failure, -3 on a HIP error.
 */
int gato_probe_lds(int pattern, int iters, double *bytes_per_clk_cu, double *bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* GATO_PROBE_H */
