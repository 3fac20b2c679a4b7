/*
 * txs_measure.h -- measurement support of the txs library (not part of the
 * method, not needed to use it).  Kernels here move the HBM traffic of a
 * method kernel in its exact layout with trivial arithmetic, so that their
 * time is the ceiling of that traffic pattern on the device, measured on the
 * same buffers the benchmark times the method kernel on.  Conventions as in
 * txs.h (device pointers owned by the caller, asynchronous on `stream`,
 * txs_status return).
 */
#ifndef TXS_MEASURE_H_
#define TXS_MEASURE_H_

#include <stddef.h>
#include <stdint.h>

#include "txs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The traffic of txs_render_bwd: reads t0, t1, sigma (float [n]) and rgb
 * (float [n,3]); writes out_a (float [n]) and out_b (float [n,3]) --
 * out_a = t0 + t1 + sigma, out_b = 2 rgb.  Arrays 16-byte aligned. */
txs_status txs_stream_probe(int64_t n_samples, const float* t0, const float* t1,
                            const float* sigma, const float* rgb, float* out_a, float* out_b,
                            void* stream);

/* The reads of txs_render_fwd: t0, t1, sigma (float [n]) and rgb (float
 * [n,3]) in its windowed layout; out (float [txs_read_probe_out_size()])
 * receives one sum per lane of every wave (it only keeps the loads live). */
int64_t txs_read_probe_out_size(void);
txs_status txs_read_probe(int64_t n_samples, const float* t0, const float* t1,
                          const float* sigma, const float* rgb, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TXS_MEASURE_H_ */
