/*
 * ensei_bench.h — comparison kernels kept out of the product library.
 *
 * libensei_bench.so (built beside libensei.so and linked against it) holds
 * the vector-ALU form of HomConv, the comparison point for the matrix-core
 * kernel that ensei_homconv runs. Benchmarks and tests load it; the product
 * path never does.
 */
#ifndef ENSEI_BENCH_H
#define ENSEI_BENCH_H

#include <stddef.h>
#include <stdint.h>

#include "ensei.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The HomConv of ensei_homconv (the Hadamard product with the transformed
 * filters, summed over input channels, plus HomShare's Delta * r on the b
 * word; Fig. 2 and Sec. 3.2) computed with 64-bit vector-ALU multiply-adds
 * straight from w_hat: uint32 [Cout][Cin][F] (values < p), one thread per
 * word. ct_in: uint64 [batch][F][n+1][Cin] (word-major), r: uint32
 * [batch][Cout][F], ct_out: uint64 [batch][F][n+1][Cout]; results are
 * bit-identical to ensei_homconv. Errors: ENSEI_ERR_ARG (null pointer,
 * non-positive size), ENSEI_ERR_LIMIT (ensei_homconv's size limits, or more
 * than 2^31 - 1 workgroups), ENSEI_ERR_ALIGN (ct 8-byte, w_hat and r 4-byte),
 * ENSEI_ERR_OVERLAP (ct_out overlapping an input), ENSEI_ERR_DEVICE, and
 * ENSEI_ERR_HIP for a launch failure; checks run before any launch. */
int ensei_bench_homconv_valu(const ensei_ctx *ctx, const uint64_t *ct_in, const uint32_t *w_hat, const uint32_t *r,
                             int64_t batch, int Cin, int Cout, int64_t F, int n, uint64_t *ct_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ENSEI_BENCH_H */
