/*
 * gcp.h -- C ABI of the MI355X (gfx950) library for the sampled stochastic
 * gradient of GCP tensor decomposition (Myers & Phipps, "Synchronous and
 * Asynchronous Parallelism Approaches for Generalized Canonical Polyadic
 * Tensor Decomposition with GenTen", arXiv 2605.20353).
 *
 * One step of GCP-SGD/Adam (Alg. gcp-sgd-iter on one device):
 *   gcp_loss_grad  -- stratified (or uniform / semi-stratified) samples of the
 *                     tensor, model values m = sum_r prod_k A_k[i_k, r]
 *                     (eq. cp), y = w f'(x, m), and the sampled MTTKRP
 *                     G_k[i_k, :] += y prod_{n != k} A_n[i_n, :]
 *                     (eq. gcp-gradient with the sampled tensor, Sec. 3.1.1-
 *                     3.1.2), all fused in one kernel;
 *   gcp_adam_step  -- Alg. adam-update over the one contiguous parameter
 *                     vector (Sec. 3.1.3).
 * GCP-FedAdam (Alg. gcp-fed-iter) runs many clients' local steps and the
 * server step in launches shared by all clients: gcp_fedadam_create /
 * gcp_fedadam_round.
 *
 * Conventions for every call:
 *   - Indices are 0-based.  Coordinates are int64, row-major [n x d].
 *   - A Kruskal model is ONE contiguous device array of sum_k I_k rows of R
 *     values, row-major, mode 0's rows first (the paper's single contiguous
 *     factor array, Sec. 3.1.3).  Gradients and Adam moments use the same
 *     layout.  No weight vector lambda: m = sum_r prod_k A_k[i_k, r].
 *   - The tensor's dtype fixes the arithmetic type of every call that uses
 *     the tensor: values x, weights w, model A, gradient G, device scale.
 *   - Device pointers are caller-owned (e.g. torch tensors passed as raw
 *     pointers) unless stated.  The library allocates device memory only in
 *     the *_create calls, never per step.
 *   - Every call is asynchronous on the given HIP stream (0 = the null
 *     stream) and returns a gcp_status.  Argument errors are found on the host
 *     before anything is launched.  Errors found inside a kernel (a zero
 *     sample that exhausted its rejection attempts, an out-of-range
 *     coordinate in a caller-supplied sample list) are recorded in a device
 *     status word and reported by gcp_device_status.  No C++ exception
 *     crosses this interface; gcp_last_error gives the calling thread's last
 *     message.
 *   - Randomness: Philox4x64-10 (Salmon et al., SC'11), key = (seed, client),
 *     counter = (s, step, stream | attempt << 8, block), stream 0 = nonzero
 *     draws, 1 = zero draws, 2 = uniform draws, block = 0 for modes 0-3 and
 *     1 for modes 4-7.  An index in [0, n) is floor(u n / 2^64) of a 64-bit
 *     output word u (exact 128-bit product).  Nonzero sample s takes
 *     j = floor(out0 N / 2^64); zero sample s tries attempts 0, 1, ... with
 *     i_k = floor(out_k I_k / 2^64) and keeps the first cell that is not a
 *     stored nonzero.  The same (seed, step, client) always yields the same
 *     samples, in gcp_sample and inside gcp_loss_grad alike.
 */
#ifndef GCP_H
#define GCP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gcp_status {
    GCP_OK = 0,
    GCP_ERR_ARG = -1,          /* invalid argument (found on the host)          */
    GCP_ERR_HIP = -2,          /* a HIP runtime call failed                     */
    GCP_ERR_OOM = -3,          /* device allocation failed (create calls only)  */
    GCP_ERR_SAMPLING = -4,     /* rejection sampling exhausted (device status)  */
    GCP_ERR_UNSUPPORTED = -5,  /* valid but not supported by this build         */
    GCP_ERR_DATA = -6          /* bad data found on the device: repeated or
                                  out-of-range coordinates                      */
} gcp_status;

typedef enum gcp_dtype { GCP_F32 = 0, GCP_F64 = 1 } gcp_dtype;

/* Losses (negative log-likelihoods, x-only terms dropped):
 *   GAUSSIAN         f = (m - x)^2 / 2,          f' = m - x
 *   POISSON          f = m - x log(m + 1e-10),   f' = 1 - x / (m + 1e-10)
 *                    (identity link; count data, the paper's experiments)
 *   BERNOULLI_LOGIT  f = log(1 + e^m) - x m,     f' = sigmoid(m) - x          */
typedef enum gcp_loss {
    GCP_LOSS_GAUSSIAN = 0,
    GCP_LOSS_POISSON = 1,
    GCP_LOSS_BERNOULLI_LOGIT = 2
} gcp_loss;

/* Sampling schemes (Sec. 3.1.1):
 *   STRATIFIED       p nonzeros with replacement, weight N/p; q zeros found by
 *                    rejection against the stored nonzeros, weight (M-N)/q.
 *   UNIFORM          p cells uniform over all M cells of a DENSE tensor,
 *                    weight M/p; q must be 0.
 *   SEMI_STRATIFIED  as STRATIFIED but zero candidates are not searched; the
 *                    nonzero samples use y = (N/p)(f'(x,m) - f'(0,m)) and the
 *                    zero samples keep weight (M-N)/q.                       */
typedef enum gcp_sampling {
    GCP_SAMPLE_STRATIFIED = 0,
    GCP_SAMPLE_UNIFORM = 1,
    GCP_SAMPLE_SEMI_STRATIFIED = 2
} gcp_sampling;

typedef struct gcp_sample_params {
    int32_t kind;          /* gcp_sampling                                       */
    int32_t max_attempts;  /* rejection attempts per zero sample; <= 0 means 64  */
    int64_t p;             /* nonzero samples (uniform: all samples)             */
    int64_t q;             /* zero samples (uniform: 0)                          */
    uint64_t seed;         /* Philox key word 0                                  */
    uint64_t step;         /* Philox counter word 1 (the iteration number)       */
    uint64_t client;       /* Philox key word 1 (0 outside GCP-FedAdam)          */
} gcp_sample_params;

/* A materialised sample list (the sampled tensor of Sec. 3.1.1), caller-owned
 * device arrays of n = p + q entries in gcp_sample's output order. */
typedef struct gcp_samples {
    const int64_t* coords; /* [n x d]                       */
    const void* x;         /* [n] tensor dtype               */
    const void* w;         /* [n] tensor dtype               */
} gcp_samples;

/* Launch shape of the sampled-gradient kernel.  Zero / negative fields take
 * the library's defaults.  A wavefront takes 64 samples at a time; each
 * sample's R columns are spread over `lanes` lanes holding `vec` consecutive
 * columns each (lanes * vec >= R, R % vec == 0). */
typedef struct gcp_tile {
    int32_t lanes;      /* 2, 4, 8, 16, 32 or 64                               */
    int32_t vec;        /* 1, 2 or 4                                           */
    int32_t block;      /* threads per workgroup, multiple of 64, <= 1024      */
    int32_t grid;       /* workgroups; 0 = sized from occupancy (ignored when
                           any mode is bucketed)                              */
    int32_t lds_modes;  /* bitmask of modes whose whole gradient is
                           accumulated in LDS per workgroup and flushed once;
                           -1 = automatic, 0 = none                           */
    int32_t bucket_modes; /* bitmask of modes scattered by row blocks (sort
                           by row, LDS accumulation per block, one flush);
                           needs gcp_tensor_reserve; -1 = automatic (every
                           mode not in LDS when a workspace is reserved and
                           p + q >= 65536), 0 = none                          */
    int32_t bucket_lds_bytes;     /* LDS bytes of one row block (rows are a
                                     power of two); 0 = 32768, min 8192     */
    int32_t bucket_block_samples; /* samples sorted per workgroup, multiple
                                     of 64 in [512, 8192]; 0 = 2048, halved
                                     while that leaves fewer than two
                                     workgroups per CU                       */
    int32_t bucket_splits;        /* workgroups per row block (each reads
                                     ceil(J / bucket_splits) of the J sort
                                     segments); 0 = auto                    */
    int32_t bucket_block;         /* threads per row-block workgroup, multiple
                                     of 64 up to 1024; 0 = 1024             */
} gcp_tile;

/* gcp_loss_grad flags */
#define GCP_LOSS_ONLY 1u        /* compute the sampled objective only          */
#define GCP_ACCUMULATE 2u       /* add into G_out / *loss_out (else overwrite) */
#define GCP_SCALE_BY_DEV 4u     /* multiply every y by *scale_dev (device
                                   scalar of the tensor dtype); the objective
                                   is not scaled                               */
#define GCP_DETERMINISTIC 8u    /* bit-identical gradient and objective on
                                   every run with the same samples, model,
                                   tile and device: the sampled tensor is
                                   written, its (row, sample) pairs sorted by
                                   row (a stable radix sort), and each gradient
                                   row with pairs summed by one lane group in
                                   the order of its sorted run;
                                   the objective's per-wavefront partial sums
                                   are added in a fixed order.  Drawn samples
                                   only (smp must be NULL); needs the workspace
                                   of gcp_tensor_reserve and (p + q) d < 2^32
                                   (GCP_ERR_ARG otherwise); slower than the
                                   default scatter                             */
/* gcp_adam_step flags */
#define GCP_ADAM_ZERO_GRAD 1u   /* write G = 0 after reading it                */

typedef struct gcp_tensor_s* gcp_tensor;
typedef struct gcp_fed_s* gcp_fed;

/* Library version string. */
const char* gcp_version(void);

/* Last error message of the calling thread ("" if none). */
const char* gcp_last_error(void);

/* sizeof of an ABI struct by name ("gcp_sample_params", "gcp_samples",
 * "gcp_tile", "gcp_fed_client", "gcp_fed_desc"), -1 if unknown: lets a
 * binding check its mirror of the layouts. */
int64_t gcp_struct_size(const char* name);

/* Sparse COO tensor (Sec. 3.1.1: N coordinate tuples and N values).
 * dims_host: d host int64 mode sizes (1 <= d <= 8 and I_k >= 1, else
 * GCP_ERR_ARG; each I_k < 2^32, sum_k I_k < 2^32 model rows and
 * prod_k I_k < 2^64 - 1 cells, else GCP_ERR_UNSUPPORTED).  coords_dev:
 * device int64 [nnz x d]; vals_dev: device values of dtype dt.  Copies and
 * packs the nonzeros into 16-byte device records {cell key, value} -- the
 * key is the bit-packed coordinates when sum_k ceil(log2 I_k) <= 63, else
 * the row-major linear index -- and builds an open-addressing hash table of
 * the keys (the O(1) membership search of Sec. 3.1.1; the smallest power of
 * two >= 4 nnz slots of 8 bytes, at least 2^10).  The inputs may be
 * freed after the call returns.  Synchronises the stream: repeated or
 * out-of-range coordinates return GCP_ERR_DATA.  The handle owns its device
 * memory until gcp_tensor_destroy. */
gcp_status gcp_tensor_create(gcp_tensor* out, int d, const int64_t* dims_host, int64_t nnz,
                             const int64_t* coords_dev, const void* vals_dev, gcp_dtype dt,
                             hipStream_t stream);

/* Dense tensor of prod_k I_k values, row-major (last mode fastest), for
 * UNIFORM sampling (dimension limits as for gcp_tensor_create).  BORROWS vals_dev: the caller keeps it alive and
 * unchanged while the handle is used. */
gcp_status gcp_tensor_create_dense(gcp_tensor* out, int d, const int64_t* dims_host,
                                   const void* vals_dev, gcp_dtype dt, hipStream_t stream);

/* Frees the handle's device memory (synchronises its device first). */
gcp_status gcp_tensor_destroy(gcp_tensor t);

/* Bytes of device memory the handle owns. */
int64_t gcp_tensor_device_bytes(gcp_tensor t);

/* Reserves the handle's workspace for the row-bucketed gradient scatter
 * (sort-by-row MTTKRP, Sec. 3.1.2) and for GCP_DETERMINISTIC calls, for calls
 * with up to max_samples = p + q samples at rank R: about 16 (max_samples +
 * 8192) d bytes of sample entries plus per-(row block, workgroup) counts, or
 * what the deterministic form needs (coordinates and derivative values of
 * the sampled tensor, (row, sample) pairs and their sort), whichever is
 * larger.  Without a reservation every large
 * mode uses hardware atomics.  Calls that use the workspace of one handle
 * must be ordered (one stream, or synchronised); concurrent calls race.
 * Replaces any earlier reservation (synchronises the device first). */
gcp_status gcp_tensor_reserve(gcp_tensor t, int64_t max_samples, int R, hipStream_t stream);

/* Synchronises the stream, then reports and clears the handle's device
 * status word: GCP_OK, GCP_ERR_SAMPLING or GCP_ERR_DATA. */
gcp_status gcp_device_status(gcp_tensor t, hipStream_t stream);

/* Materialises the sample list (Sec. 3.1.1): n = p + q samples, the p
 * nonzero samples first.  coords_out [n x d] int64, x_out [n] and w_out [n]
 * of the tensor dtype, all device, caller-owned.  Bit-exact reproducible. */
gcp_status gcp_sample(gcp_tensor t, const gcp_sample_params* sp, int64_t* coords_out,
                      void* x_out, void* w_out, hipStream_t stream);

/* Sampled objective and gradient, fused (Sec. 3.1.2 "Fused Sampling-MTTKRP",
 * here with stratified, uniform or semi-stratified sampling).
 *   smp == NULL: the samples of `sp` are drawn inside the kernel and never
 *                stored (identical to what gcp_sample returns for `sp`);
 *   smp != NULL: the materialised list is read instead (sp->kind and sp->p
 *                still say which entries are semi-stratified nonzeros).
 * A: device model [sum_k I_k x R]; R <= 64, or even R <= 128, or R <= 256
 * divisible by 4 (GCP_ERR_ARG otherwise).  G_out: device gradient of
 * the same shape (may be NULL with GCP_LOSS_ONLY).  loss_out: device double
 * receiving F~ = sum_s w_s f(x_s, m_s) (NULL = not computed).  Unless
 * GCP_ACCUMULATE is set, G_out and *loss_out are overwritten.  tile: launch
 * shape (NULL = defaults).  Duplicate samples are summed as separate entries;
 * atomics make the summation order unspecified. */
gcp_status gcp_loss_grad(gcp_tensor t, const gcp_sample_params* sp, const gcp_samples* smp,
                         const void* A, int R, gcp_loss loss, unsigned flags,
                         const void* scale_dev, void* G_out, double* loss_out,
                         const gcp_tile* tile, hipStream_t stream);

/* The non-fused sampled gradient (Sec. 3.1.2, the form the "Fused
 * Sampling-MTTKRP" paragraph improves on): the sampling step computes every
 * sample's model value and derivative and stores the sampled tensor Y~, and
 * a separate MTTKRP reads Y~ and gathers the factor rows a second time.
 *
 * gcp_sample_y draws the samples of `sp` exactly as gcp_sample does, gathers
 * their factor rows, and writes coords_out [n x d] (int64, device) and
 * y_out [n] (tensor dtype, device) with y_s = w_s f'(x_s, m_s) (semi-
 * stratified nonzero samples: w_s (f'(x_s, m_s) - f'(0, m_s))); loss_out
 * (device double, nullable) receives F~ as in gcp_loss_grad.  Nothing is
 * scattered; tile may set the lane shape and block (its scatter fields are
 * ignored).  Errors as gcp_loss_grad; NULL coords_out or y_out is
 * GCP_ERR_ARG. */
gcp_status gcp_sample_y(gcp_tensor t, const gcp_sample_params* sp, const void* A, int R, gcp_loss loss,
                        int64_t* coords_out, void* y_out, double* loss_out, const gcp_tile* tile,
                        hipStream_t stream);

/* Sampled MTTKRP of a given sampled tensor (eq. gcp-gradient with Y~):
 *   G_k[i_k(s), :] += y_s prod_{j != k} A_j[i_j(s), :]   for every mode k,
 * over the n entries of coords [n x d] (int64, device, each coordinate in
 * range, else GCP_ERR_DATA through gcp_device_status) and y [n] (tensor
 * dtype, device).  t supplies the dims and, when reserved, the row-bucketing
 * workspace.  flags: GCP_ACCUMULATE (else G_out is overwritten) and
 * GCP_SCALE_BY_DEV (every y times *scale_dev); tile as gcp_loss_grad (the
 * same scatter strategies).  Duplicates are summed; the order of additions is
 * unspecified. */
gcp_status gcp_mttkrp(gcp_tensor t, int64_t n, const int64_t* coords, const void* y, const void* A, int R,
                      unsigned flags, const void* scale_dev, void* G_out, const gcp_tile* tile,
                      hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as gcp_loss_grad, with the same arguments, results and errors, except
 * that the row-bucketed scatter uses the library's own fixed scratch region of
 * gcp_noalloc_scratch_bytes() bytes (128 MiB) per GPU instead of the
 * handle's gcp_tensor_reserve workspace, and no call allocates or frees device
 * memory.  A call needs nblocks * spb * b * 16 + nbk * nblocks * 8 bytes of it
 * (spb samples per sorting workgroup, nblocks = ceil((p + q) / spb), b
 * bucketed modes, nbk row blocks over those modes); that is 97 MiB for 2^21
 * samples of a 10000 x 8000 x 6000 tensor at rank 32 in float32.  With
 * tile->bucket_modes = -1 (automatic) a call whose need exceeds the scratch
 * uses hardware atomics instead; an explicit bucket_modes request that does
 * not fit returns GCP_ERR_ARG.  The first call on a device looks up the
 * scratch region's address there; each GPU keeps its copy until the process
 * ends.  All calls on one GPU share its copy: calls that overlap in time on
 * one GPU (different streams, or different host threads without ordering)
 * race and give wrong gradients; calls ordered on one stream are safe. */
gcp_status gcp_loss_grad_noalloc(gcp_tensor t, const gcp_sample_params* sp, const gcp_samples* smp,
                                 const void* A, int R, gcp_loss loss, unsigned flags,
                                 const void* scale_dev, void* G_out, double* loss_out,
                                 const gcp_tile* tile, hipStream_t stream);

/* Size in bytes of the per-GPU scratch region of gcp_loss_grad_noalloc. */
int64_t gcp_noalloc_scratch_bytes(void);

/* Alg. adam-update on n contiguous parameters of dtype dt, one launch:
 *   B = b1 B + (1-b1) G;  C = b2 C + (1-b2) G*G;
 *   A = max(A - lr (B/(1-b1^t)) / sqrt(C/(1-b2^t) + eps), lower)
 * (epsilon inside the square root, as the paper writes it; lower = -INFINITY
 * disables the bound).  t >= 1 is this model's update count.  A, B, C are
 * updated in place; G is read (and zeroed with GCP_ADAM_ZERO_GRAD). */
gcp_status gcp_adam_step(void* A, void* G, void* B, void* C, int64_t n, gcp_dtype dt, int64_t t,
                         double lr, double beta1, double beta2, double eps, double lower,
                         unsigned flags, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* GCP-FedAdam (Alg. gcp-fed-iter): K clients, each holding one block of a   */
/* d-way block grid over the tensor, run tau local GCP-Adam steps on their   */
/* own model; then the server model takes one Adam step whose gradient is    */
/* the per-row mean of the deltas D = U - M_c over the clients whose block   */
/* covers the row (the all-reduce over slice groups, here within one GPU).   */
/* One round (gcp_fedadam_round with round r) is:                            */
/*   1. M_c <- rows of U covered by client c, for every c;                    */
/*   2. tau local steps j = 0..tau-1 per client: stratified samples of the    */
/*      client's block with Philox key (seed, c) and step r*tau + j, sampled  */
/*      gradient into G_c, Adam on (M_c, B_c, C_c) with t = r*tau + j + 1;     */
/*   3. D = per-row mean over covering clients of U - M_c;                    */
/*   4. Adam on (U, B_s, C_s) with gradient D, lr = meta_lr, t = r + 1.       */
/* Client moments persist across rounds; only M_c is reset to U.            */
/* ------------------------------------------------------------------------ */

typedef struct gcp_fed_client {
    gcp_tensor tensor;        /* the client's block, block-local coordinates       */
    int64_t row_base[8];      /* global index of the block's first row, per mode   */
    void* M;                  /* client model [sum_k I_k^c x R], device            */
    void* B;                  /* client Adam moments, same shape                   */
    void* C;
    void* G;                  /* client gradient buffer, same shape; must hold
                                 zeros before the first round (it is left zeroed
                                 after every round)                               */
} gcp_fed_client;

typedef struct gcp_fed_desc {
    int32_t nclients;         /* K >= 1                                           */
    int32_t R;                /* rank                                             */
    int32_t tau;              /* local steps per round >= 1                       */
    int32_t loss;             /* gcp_loss                                         */
    int32_t batched;          /* 1: every client's local steps run in shared
                                 launches over all clients (one persistent launch
                                 per round, or three row-bucketed launches per
                                 local step, see bucket_modes); 0: one sampled-
                                 gradient launch and one Adam launch per client
                                 and local step                                  */
    int32_t use_graph;        /* batched only: capture the round's launches into
                                 a HIP graph on the first round, replay after     */
    int32_t workgroups_per_client; /* batched launch shape; 0 = automatic: the
                                 persistent launch takes as many as stay
                                 resident over K clients, at most enough for
                                 about four 64-sample chunks per wavefront of
                                 a local step; the row-bucketed sampling
                                 launch as many as stay resident, at most one
                                 per sample block                                */
    int32_t block;            /* threads per workgroup (batched), 0 = 256 (1024
                                 for row-bucketed rounds)                         */
    int32_t lanes;            /* lane shape of the gradient part, 0 = default    */
    int32_t vec;
    int32_t max_attempts;     /* rejection attempts per zero sample, <= 0 = 64   */
    int32_t lds_modes;        /* batched: bitmask of modes whose client gradient
                                 is accumulated in each workgroup's LDS and
                                 flushed once per local step; -1 = automatic
                                 (modes whose largest client block fits), 0 = none */
    int32_t bucket_modes;     /* per-client rounds: passed as tile.bucket_modes
                                 to every gcp_loss_grad call (-1 = that call's
                                 automatic choice, which row-buckets only when
                                 the client tensor has a gcp_tensor_reserve
                                 workspace, and with lanes and vec left 0 also
                                 its own lane shape; 0 = hardware atomics).
                                 batched: bitmask of modes scattered by the row-
                                 bucketed (sort-by-row) scheme inside the launch:
                                 each client's workgroups sort their samples by
                                 row block, then each owns whole row blocks and
                                 writes them without atomics (modes that are
                                 LDS-private are left out).  Such rounds run as
                                 three launches per local step over all clients
                                 (sample and sort, row-block owners, Adam)
                                 instead of the persistent launch; default
                                 block 1024 and, in FP32, four columns per lane.
                                 -1 = automatic: every mode that is not LDS-
                                 private at >= 2^14 samples per client step,
                                 else none; 0 = none (hardware atomics)         */
    int32_t bucket_block_samples; /* samples per sorted block, multiple of 64 in
                                 [512, 8192]; 0 = 2048                            */
    int64_t p;                /* nonzero samples per client and local step       */
    int64_t q;                /* zero samples per client and local step          */
    uint64_t seed;
    int64_t global_dims[8];   /* d = the clients' tensor order                   */
    void* U;                  /* server model [sum_k I_k x R], device            */
    void* Bs;                 /* server Adam moments, same shape                 */
    void* Cs;
    double lr;                /* client Adam rate                                 */
    double meta_lr;           /* server Adam rate (meta-rate)                     */
    double beta1, beta2, eps, lower;   /* shared by client and server Adam       */
    const gcp_fed_client* clients;     /* host array of nclients entries         */
    double barrier_timeout_s; /* persistent launch: a group barrier that waits
                                 longer than this (device wall clock) gives up
                                 and fails the round; <= 0 = 10 s              */
} gcp_fed_desc;

/* How a handle runs its rounds (gcp_fedadam_info). */
typedef enum gcp_fed_form {
    GCP_FED_PER_CLIENT = 0,   /* per client and local step: one gcp_loss_grad
                                 and one gcp_adam_step launch                */
    GCP_FED_PERSISTENT = 1,   /* one persistent launch for every client and
                                 local step (group barriers), hardware atomics
                                 or LDS-private scatter                      */
    GCP_FED_ROW_BUCKETED = 2  /* per local step three launches over all
                                 clients: sample and sort by row block, row-
                                 block owners, Adam                          */
} gcp_fed_form;

typedef struct gcp_fed_info {
    int32_t form;                 /* gcp_fed_form                                  */
    int32_t lds_modes;            /* batched: modes accumulated in LDS per
                                     workgroup; per-client: the request (-1 =
                                     decided per launch)                        */
    int32_t bucket_modes;         /* batched: row-bucketed modes; per-client: the
                                     request passed to every gcp_loss_grad       */
    int32_t workgroups_per_client;/* batched                                      */
    int32_t block, lanes, vec;    /* launch shape of the gradient part (0: each
                                     call's own choice)                         */
    int32_t bucket_block_samples; /* row-bucketed form: samples per sorted block */
    int64_t launches_per_round;   /* kernel launches one round issues (per-client
                                     rounds that may row-bucket: at most)        */
} gcp_fed_info;

/* Validates the description, copies it, and builds the device-side client
 * table and the row-coverage table of the server step.  Every buffer stays
 * caller-owned; the tensors must outlive the handle.  The clients' blocks
 * must lie inside global_dims.  A batched handle needs all its workgroups
 * resident at once (K * workgroups_per_client <= what the GPU holds):
 * GCP_ERR_UNSUPPORTED otherwise. */
gcp_status gcp_fedadam_create(gcp_fed* out, const gcp_fed_desc* desc, hipStream_t stream);

/* Runs round `round` (see above) asynchronously on the stream.  Batched
 * rounds are either one persistent kernel for all clients and tau steps
 * (GCP_FED_PERSISTENT) or three launches over all clients per local step
 * (GCP_FED_ROW_BUCKETED), then one server kernel; with use_graph the round's
 * launches are captured into a HIP graph on the first round and replayed
 * after (the graph is bound to the stream of its first capture).  The
 * persistent kernel's group barriers give up after barrier_timeout_s of
 * device wall clock instead of hanging: the status records GCP_ERR_HIP, the
 * rest of that round (local steps and the server step) is skipped, and every
 * later round does nothing until gcp_fedadam_status clears the status.  A
 * round launched after such a failure has been copied back to the host
 * returns GCP_ERR_HIP at once, without launching. */
gcp_status gcp_fedadam_round(gcp_fed f, int64_t round, hipStream_t stream);

/* Synchronises the stream; reports a barrier timeout of a batched round
 * (GCP_ERR_HIP) or a sampling error of any client tensor (GCP_ERR_SAMPLING),
 * and clears them. */
gcp_status gcp_fedadam_status(gcp_fed f, hipStream_t stream);

/* Fills *out with how the handle runs its rounds (form, scatter modes,
 * launch shape).  Host only. */
gcp_status gcp_fedadam_info(gcp_fed f, gcp_fed_info* out);

/* Frees the handle (its graph and device tables; not the caller's buffers). */
gcp_status gcp_fedadam_destroy(gcp_fed f);

#ifdef __cplusplus
}
#endif

#endif /* GCP_H */
