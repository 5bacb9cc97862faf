/*
 * gcp_ceilings.h -- microbenchmarks of the MI355X ceilings that bound the
 * sampled stochastic gradient of GCP decomposition (the access patterns of
 * Sec. 3.1.1-3.1.2 taken one at a time: random reads of tensor records,
 * dependent factor-row gathers, LDS compare-and-swap accumulation, global
 * float atomics, streaming copies).  Measurement tools, part of libgcp.so;
 * none computes anything of the method.  Each call launches one kernel,
 * asynchronously on the stream, sized to fill the device; the caller times
 * it (HIP events) and owns every buffer.  Errors: GCP_ERR_ARG for bad
 * arguments (checked on the host, nothing launched), GCP_ERR_HIP when the
 * launch fails.
 */
#ifndef GCP_CEILINGS_H
#define GCP_CEILINGS_H

#include "gcp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* nreads independent 16-byte loads at pseudo-random positions of rec, a
 * device array of nrec 16-byte records; in_flight (1 or 4) loads issued per
 * lane before their results are used; block threads per workgroup (multiple
 * of 64, <= 1024).  sink: device scratch of >= 4096 bytes (practically never
 * written). */
gcp_status gcp_ceiling_random_reads(const void* rec, int64_t nrec, int64_t nreads, int in_flight, int block,
                                    void* sink, hipStream_t stream);

/* nsamples times: one 16-byte record of rec (nrec records; pseudo-random,
 * or with sequential != 0 the next of a stream), then, from a hash of its
 * contents, one row in each of three modes of dims3[0], dims3[1], dims3[2]
 * (each < 2^30) rows of A (device float array of (dims3[0] + dims3[1] +
 * dims3[2]) x 32), gathered by eight lanes of four floats, two samples in
 * flight per lane group.  sink: device scratch of >= 4096 bytes. */
gcp_status gcp_ceiling_dependent_gathers(const void* rec, int64_t nrec, const float* A, const int64_t* dims3,
                                         int64_t nsamples, int sequential, int block, void* sink,
                                         hipStream_t stream);

/* grid workgroups of block threads, each lane doing iters 64-bit LDS
 * compare-and-swap float-pair adds into its own words (block * 32 bytes of
 * LDS per workgroup).  sink: device scratch of >= 4 * grid bytes. */
gcp_status gcp_ceiling_lds_cas(int iters, int block, int grid, void* sink, hipStream_t stream);

/* grid workgroups of 1024 threads, each with an LDS block of 256 rows x 32
 * values; every iteration each group of 8 lanes picks a row at random and
 * each lane adds 4 values to its 4 columns (4 * iters adds per lane).
 * form 0: float block (32 KB), two 64-bit compare-and-swap float-pair loops
 * per lane; form 1: float block, four native LDS float atomic adds; form 2:
 * double block (64 KB), four native LDS double atomic adds.  sink: device
 * scratch of >= 4 * grid bytes. */
gcp_status gcp_ceiling_lds_row_adds(int form, int iters, int grid, void* sink, hipStream_t stream);

/* nupdates requests of 32 float atomic adds (one 128-byte row) at
 * pseudo-random rows of G, a device array of rows x 32 floats (modified). */
gcp_status gcp_ceiling_global_atomics(float* G, int64_t rows, int64_t nupdates, int block, hipStream_t stream);

/* Device-to-device copy of bytes (a multiple of 16) with float4 loads and
 * stores. */
gcp_status gcp_ceiling_copy(const void* src, void* dst, int64_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GCP_CEILINGS_H */
