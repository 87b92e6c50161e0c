/*
 * lic.h - C ABI of the MI355X learned-image-codec library.
 *
 * The library implements the streaming architecture for learned image codecs
 * of Lin, Sun and Katto (arXiv 2208.01641): an encoder takes frames and
 * produces bitstreams ("strings"), a decoder takes bitstreams and produces
 * frames (Section III.A-B).  The neural transforms (g_a, h_a, h_s, g_s with
 * GDN/IGDN, quantisation and the scale-table index) run as HIP kernels on
 * one GPU; rANS entropy coding runs on CPU worker threads; the two are
 * overlapped in a multi-stage pipeline with pooled, pinned host buffers
 * (Sections III.A-D: 2-stage encoder, 2-stage factorized decoder, 4-stage
 * hyperprior decoder CPU1-GPU1-CPU2-GPU2, zero-copy memory with a toggle,
 * memory pooling).  Every frame is an independent keyframe (Section VI).
 *
 * Conventions
 *   - Every call returns a lic_status (0 = success, negative = error); no
 *     exception or abort crosses the ABI.  codec_last_error() gives a message.
 *   - The caller owns every input and output buffer; the codec owns its HIP
 *     streams, device memory pool, pinned host slots, threads and tables.
 *   - A codec handle is used by one calling thread at a time.
 *   - Images are n x 3 x H x W float32 (NCHW) in [0, 1].  H and W need not be
 *     multiples of 64: frames are zero-padded at the bottom/right to the next
 *     multiple of 64 inside the codec and decoded frames are cropped back.
 *   - Pointers flagged "is_device" are HIP device pointers on the codec's
 *     device; the caller must have completed all work producing them before
 *     the call (the library runs on its own streams).
 */
#ifndef LIC_H
#define LIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct codec codec_t;

typedef enum {
    LIC_OK = 0,
    LIC_E_ARG = -1,       /* invalid argument or unsupported configuration        */
    LIC_E_NOMEM = -2,     /* host or device allocation failed (at create only)    */
    LIC_E_HIP = -3,       /* a HIP runtime call failed                            */
    LIC_E_CORRUPT = -4,   /* malformed, truncated or inconsistent bitstream       */
    LIC_E_SMALLBUF = -5,  /* output capacity too small; required sizes returned   */
    LIC_E_BUDGET = -6,    /* request exceeds the configured limits (size/memory)  */
    LIC_E_STATE = -7,     /* call not valid in the codec's current state          */
    LIC_E_MODEL = -8      /* weight blob or bitstream belongs to another model    */
} lic_status;

enum { LIC_KIND_FACTORIZED = 0, LIC_KIND_HYPERPRIOR = 1,
       LIC_KIND_CONTEXT = 2 };  /* mean-scale hyperprior with a checkerboard context model */
enum { LIC_PREC_FP32 = 0, LIC_PREC_BF16 = 1, LIC_PREC_FP8 = 2 };
enum { LIC_HS_RELU = 0, LIC_HS_EXP = 1 };
enum { LIC_NORM_GDN = 0, LIC_NORM_1DN = 1 };

/* Creation parameters.  Fill with codec_default_config() first. */
typedef struct {
    uint32_t struct_size;      /* sizeof(codec_config), for ABI versioning           */
    int32_t  kind;             /* LIC_KIND_*: factorized prior [1], hyperprior [2],  */
                               /* or the context model: a mean-scale hyperprior      */
                               /* whose entropy parameters also see a context of     */
                               /* decoded latents, in two parallel checkerboard      */
                               /* passes (the parallel context prediction Sections   */
                               /* II and VII point to; N=128 M=192, any precision   */
                               /* form, full g_s, no serving; its h_a / h_s, context */
                               /* and entropy-parameter layers run in FP32; its      */
                               /* symbols and indices go through device buffers and  */
                               /* copies whatever zero_copy says)                    */
    int32_t  N, M;             /* transform / latent channels (128/192 or 192/320)   */
    int32_t  precision;        /* LIC_PREC_FP32, _BF16 or _FP8: g_a / g_s GEMM       */
                               /* operands and their activations in bf16, or in OCP  */
                               /* e4m3 with per-output-channel FP32 weight scales    */
                               /* and per-layer activation scales (codec_calibrate;  */
                               /* the image layer, g_s's first and last layers run   */
                               /* on bf16 operands in that form; FP32 accumulation;  */
                               /* GDN/IGDN normaliser from three bf16 part products, */
                               /* about 2^-16 relative, normalisation in FP32);      */
                               /* h_a, h_s, the quantisers and the scale index stay  */
                               /* FP32                                               */
    int32_t  hs_out;           /* output activation of h_s: LIC_HS_EXP or _RELU      */
    int32_t  gs_mode;          /* 0: full synthesis transform g_s; 1: distilled g_s  */
                               /* (codec_load_distilled); 2: distilled g_s with a    */
                               /* sampled judge that falls back to the full g_s      */
    int32_t  y_slices;         /* S >= 1 independent rANS streams for y (row bands)  */
    int32_t  entropy_threads;  /* CPU entropy worker threads (paper: 3 and 10)       */
    int32_t  zero_copy;        /* 1: kernels read/write mapped pinned host slots;    */
                               /* 0: device buffers plus async copies (Sec. III.D)   */
    int32_t  max_in_flight;    /* frames in flight = pooled slots per pipeline       */
    int32_t  max_h, max_w;     /* largest frame the pools are sized for              */
    int32_t  max_batch;        /* frames per task = per GPU launch (1..8)            */
    uint64_t hbm_budget_bytes; /* device memory the codec may take: pools plus the   */
                               /* reservations of open serving streams (0 = no limit)*/
    int32_t  hip_device;       /* HIP device ordinal                                 */
    int32_t  use_graphs;       /* serving: run each GPU stage of a (frame size,      */
                               /* batch, slot) as a captured HIP graph               */
    int32_t  norm;             /* normalisation of g_a / g_s (Section IV.C):         */
                               /* LIC_NORM_GDN y_i = x_i / sqrt(beta_i + sum_j       */
                               /* gamma_ij x_j^2), inverse x_i sqrt(...); or         */
                               /* LIC_NORM_1DN (implementation C, whose formula the  */
                               /* paper does not print; read as) y_i = x_i /         */
                               /* (beta_i + sum_j gamma_ij |x_j|), inverse x_i (...) */
                               /* with the same beta / gamma; recorded in streams    */
    int32_t  rans_lanes;       /* entropy coder: 0 byte-wise rANS with one state;    */
                               /* 2, 4, 8, 16 or 32: interleaved word-wise rANS with */
                               /* that many states (lic_rans_ileave_encode); recorded */
                               /* in streams                                         */
} codec_config;

/* Defaults: hyperprior, N=128, M=192, FP32, exp output, S=8, 8 entropy
 * threads, zero_copy=1, 6 tasks in flight, 1088x1920 max, batch 1, graphs on,
 * GDN, byte-wise rANS. */
void codec_default_config(codec_config* cfg);

/* Creates a codec from a "LICW" weight blob (see DESIGN notes: per-layer
 * float32 weights in PyTorch layouts, GDN beta/gamma, float64 raw density
 * parameters).  The blob's kind/N/M must match cfg (else LIC_E_MODEL).  The
 * blob is copied; the caller may free it after the call.  Builds all entropy
 * tables, uploads packed weights, allocates every pool.  *out = NULL on error. */
int codec_create(const codec_config* cfg, const void* weight_blob, size_t blob_len, codec_t** out);

/* Encodes n frames (pipelined).  x: n x 3 x H x W float32, host or device.
 * Bitstreams are written back to back into out[0..cap); lens[i] receives the
 * length of frame i.  On LIC_E_SMALLBUF lens[] holds each frame's size and
 * the contents of out are unspecified. */
int codec_encode(codec_t* c, const float* x, int n, int H, int W, int is_device,
                 uint8_t* out, size_t cap, size_t* lens);

/* Decodes n bitstreams stored back to back in bits (lengths lens[0..n)).
 * All frames must share one size; *H, *W receive it.  x_hat receives
 * n x 3 x H x W float32 (host or device) and holds cap_elems floats. */
int codec_decode(codec_t* c, const uint8_t* bits, const size_t* lens, int n,
                 float* x_hat, size_t cap_elems, int is_device, int* H, int* W);

/* Encoder chained into the decoder per frame (one pipeline: GPU encode, CPU
 * encode, CPU1, GPU1, CPU2, GPU2 for the hyperprior).  Writes the bitstreams
 * like codec_encode and the reconstructions like codec_decode. */
int codec_encode_decode(codec_t* c, const float* x, int n, int H, int W, int is_device,
                        uint8_t* bits, size_t cap, size_t* lens, float* x_hat);

/* Per-frame latency (milliseconds, admission to result ready) of the last
 * encode / decode / encode_decode call, in frame order.  Returns the count
 * written (at most max). */
int codec_last_latencies(const codec_t* c, double* ms, int max);

/* JSON statistics of the last call (frames/s, p50/p99, per-stage busy time). */
int codec_get_stats(const codec_t* c, char* buf, size_t cap);

/* Drains in-flight work, joins threads, frees pools.  NULL-safe. */
void codec_destroy(codec_t* c);

/* Message describing the last error on this handle (valid until the next
 * call on it).  With c == NULL: the last error of a failed codec_create. */
const char* codec_last_error(const codec_t* c);

/* ------------------------------------------------------------------------ */
/* Serving: many concurrent streams of mixed frame sizes (Section VI's       */
/* streaming use, many cameras to one server).  Requests queue per          */
/* (direction, frame size) bucket; whenever a pool slot frees up, up to     */
/* max_batch queued requests of the bucket that has waited longest are      */
/* admitted as one task and share every GPU launch, while earlier tasks are */
/* still on the GPU or the entropy workers (continuous batching).  With     */
/* use_graphs each GPU stage of a (frame size, batch, slot) runs as a       */
/* captured HIP graph.  A request's result is bit-identical alone and in a  */
/* batch.  Results come back through codec_poll in completion order.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t ticket;
    int32_t  status;      /* lic_status of the request                          */
    int32_t  stream_id;
    int32_t  direction;   /* 0 encode, 1 decode                                 */
    int32_t  H, W;
    uint64_t bytes;       /* encode: bitstream length                           */
    double   latency_ms;  /* submit to result ready                             */
} lic_result;

/* Admits a stream of H x W frames: reserves its device footprint (one frame
 * in flight: input, reconstruction and the two largest activations) against
 * hbm_budget_bytes.  LIC_E_BUDGET if it does not fit or exceeds max_h x max_w. */
int codec_open_stream(codec_t* c, int H, int W, int* stream_id);
/* Releases the reservation; requests already queued still complete. */
int codec_close_stream(codec_t* c, int stream_id);
/* Queues one frame (3 x H x W float32 at the stream's size) for encoding;
 * the bitstream goes to out[0..cap) (status LIC_E_SMALLBUF if it does not
 * fit).  x and out must stay valid until the result is polled. */
int codec_submit_encode(codec_t* c, int stream_id, const float* x, int is_device,
                        uint8_t* out, size_t cap, uint64_t* ticket);
/* Queues one bitstream (validated now) for decoding into x_hat
 * (3 x H x W float32).  bits and x_hat must stay valid until polled. */
int codec_submit_decode(codec_t* c, int stream_id, const uint8_t* bits, size_t len,
                        float* x_hat, size_t cap_elems, int is_device, uint64_t* ticket);
/* Waits up to timeout_us for completed requests; returns the number written
 * to done (0 on time-out). */
int codec_poll(codec_t* c, lic_result* done, int max, int timeout_us);

/* ------------------------------------------------------------------------ */
/* Stage-level entry points: one layer of the transforms on device buffers,  */
/* run synchronously on the codec's stream.  For parity checks and           */
/* profiling.  H, W are the original frame size; the layer's tensor sizes    */
/* follow from the 64-multiple padded size Hp x Wp (latents Hp/16 x Wp/16,   */
/* hyper-latents Hp/64 x Wp/64).  All tensors are NHWC except images.        */
/*                                                                          */
/*  In the BF16 form the NHWC activations in and out of GA0..GA2 and       */
/*  GS0..GS2 (and into GA3 / GS3) are bf16; in the FP8 form they are e4m3   */
/*  bytes (8 x value) except GS2's output (into GS3), bf16; y, z, v and     */
/*  images stay f32.  codec_layer_bytes gives every buffer's size.          */
/*  layer          in                         out                aux         */
/*  LIC_GA0..GA2   ga0: image NCHW f32         NHWC f32           -           */
/*  LIC_GA3        NHWC f32                    y NHWC f32         sym_y int8  */
/*  LIC_HA0..HA1   NHWC f32 (ha0 takes y)      NHWC f32           -           */
/*  LIC_HA2        NHWC f32                    z NHWC f32         sym_z int8  */
/*  LIC_HS0        sym_z int8 NHWC             NHWC f32           -           */
/*  LIC_HS1        NHWC f32                    NHWC f32           -           */
/*  LIC_HS2        NHWC f32                    idx uint8 NHWC     v f32 / NULL*/
/*  LIC_GS0        sym_y int8 NHWC             NHWC f32           -           */
/*  LIC_GS1..GS2   NHWC f32                    NHWC f32           -           */
/*  LIC_GS3        NHWC f32                    image NCHW f32 (cropped,      */
/*                                             clamped)           pre-clamp   */
/*                                             image n x 3 x Hp x Wp / NULL   */
/*                                                                          */
/*  Context model (kind 2; every tensor on the Hy x Wy latent grid, f32):   */
/*  HA0 takes y itself; HS2 writes psi (2M channels) into channels [0, 2M)  */
/*  of Z = [psi; ctx] (4M channels); GS0 takes y_hat (f32, bf16 in the BF16  */
/*  form).  The anchors are the positions with (row + column) even; the     */
/*  *A layers run at the anchors, the *N layers at the other positions.     */
/*  LIC_CX         y_hat NHWC (anchors read)   Z, channels [2M, 4M) at the   */
/*                                             non-anchors (checkerboard-    */
/*                                             masked 5x5 convolution)        */
/*  LIC_EP0A/N     Z                           h1 NHWC (640 ch)   -           */
/*  LIC_EP1A/N     h1                          h2 NHWC (512 ch)   -           */
/*  LIC_EP2A/N     h2                          idx uint8          sym int8 /  */
/*                                                                NULL        */
/*    with codec_run_layer_ex: in2 = y (encoder) or NULL (decoder); out2 =  */
/*    y_hat = sym + mean on the full grid (encoder) or the means (decoder). */
/*    idx, sym and the decoder's means are checkerboard-major: [n][part]    */
/*    [Hy][Wy/2][M], part 0 the anchors, entry j of row r at column         */
/*    2j + ((r + part) & 1).  The anchors' ctx channels of Z must be zero   */
/*    (the codec clears them; a caller of EP0A does).                       */
/* ------------------------------------------------------------------------ */
enum {
    LIC_GA0 = 0, LIC_GA1, LIC_GA2, LIC_GA3,
    LIC_HA0, LIC_HA1, LIC_HA2,
    LIC_HS0, LIC_HS1, LIC_HS2,
    LIC_GS0, LIC_GS1, LIC_GS2, LIC_GS3,
    /* context model (kind 2) */
    LIC_CX,                           /* context convolution of the non-anchors */
    LIC_EP0A, LIC_EP1A, LIC_EP2A,     /* entropy parameters, anchor pass */
    LIC_EP0N, LIC_EP1N, LIC_EP2N,     /* entropy parameters, second pass */
    LIC_NUM_LAYERS
};
/* Loads the distilled synthesis transform used by the decoder when gs_mode
 * is 1 or 2 (parameters as for lic_distill_create, M of this codec, F = 64,
 * host array, copied; GEMM operands in the codec's precision).  With gs_mode
 * 2, the task holding every judge_every-th decoded frame also decodes its
 * first frame with the full g_s; if PSNR(full, distilled) < judge_psnr_db
 * the codec switches to the full g_s for good (the judged task included).
 * codec_get_stats reports gs_judged, gs_judge_last_db and gs_fallback.  Call
 * while no decode is in flight. */
int codec_load_distilled(codec_t* c, const float* params, size_t n_params, float judge_psnr_db,
                         int judge_every);

/* FP8 form: sets the activation scale of every layer that stores e4m3
 * activations from calibration frames x (n x 3 x H x W float32 in [0, 1],
 * host or device): the layer's activations are stored as e4m3(q * value)
 * with q = 448 / (2 amax), amax the largest |value| the layer produces on
 * these frames (layers calibrated in order, each with its predecessors'
 * scales in place); the reading layer undoes q in its epilogue.  Until the
 * first call every q is 8.  Other forms: no effect.  Encoders and decoders
 * must use the same scales for identical reconstructions (the bitstream does
 * not carry them).  Call while no work is in flight; captured serving graphs
 * are dropped. */
int codec_calibrate(codec_t* c, const float* x, int n, int H, int W, int is_device);
/* FP8 form: q of each layer (LIC_NUM_LAYERS entries; 0 for layers that do
 * not store e4m3) and, if saturated != NULL, the number of values the e4m3
 * stores have clamped to +-448 since create.  Returns LIC_NUM_LAYERS. */
int codec_fp8_scales(const codec_t* c, float* q, int max, unsigned long long* saturated);

int codec_run_layer(codec_t* c, int layer, int n, int H, int W,
                    const void* in, void* out, void* aux);
/* The same with the second input and output of LIC_EP2A / LIC_EP2N (see the
 * table above); other layers ignore in2 and out2. */
int codec_run_layer_ex(codec_t* c, int layer, int n, int H, int W, const void* in, void* out, void* aux,
                       const void* in2, void* out2);
/* Bytes codec_run_layer reads from in and writes to out / aux for n frames
 * of H x W in this codec's form (0: the layer takes no such buffer; aux is
 * optional where the table above says so).  Element sizes: images, y, z,
 * v and the hyper activations float32, symbols int8, indices uint8, the
 * GDN layers' activations float32 (FP32 form), bf16 (BF16 form), or e4m3
 * (FP8 form; GS2 stores bf16 there, read by GS3 on bf16 operands). */
int codec_layer_bytes(codec_t* c, int layer, int n, int H, int W, size_t* in_bytes,
                      size_t* out_bytes, size_t* aux_bytes);

/* Kernel timing inside the pipeline: every launch of a layer whose bit is
 * set in mask (bit i = layer i) is bracketed with HIP events on the stream
 * it runs on; the accumulators are reset.  codec_layer_time returns the
 * summed kernel time (ms) and launch count of one layer since then. */
int codec_time_layers(codec_t* c, uint32_t mask);

/* Which kernel a layer launches for one H x W frame (nothing is launched):
 * *form = the operand form of its GEMM (LIC_FORM_*), *ksplit = the number of
 * waves that split its K loop (1: one wave per pixel tile).  The choice
 * depends on the codec's precision and the frame size only. */
enum { LIC_FORM_F32 = 0,     /* FP32 operands on the FP32 matrix cores */
       LIC_FORM_BF16 = 1,    /* bf16 operands */
       LIC_FORM_FP8 = 2,     /* OCP e4m3 operands, per-row weight scales */
       LIC_FORM_F32X = 3 };  /* FP32 operands as three exact bf16 parts: six
                                bf16 products per FP32 product, FP32 sums */
int codec_layer_kernel(codec_t* c, int layer, int H, int W, int* form, int* ksplit);
int codec_layer_time(codec_t* c, int layer, double* total_ms, long* launches);

/* Entropy tables the codec built at create (host copies, for checking):
 * which 0 = factorized tables [C][129] (C = N for the hyperprior's z, M for
 * the factorized prior's y), 1 = Gaussian tables [64][129].  Returns the
 * number of uint32 written, or LIC_E_SMALLBUF.  Channel offsets (medians,
 * float32) via codec_medians. */
long codec_tables(const codec_t* c, int which, uint32_t* freq, size_t cap);
long codec_medians(const codec_t* c, float* mu, size_t cap);

/* ------------------------------------------------------------------------ */
/* Distilled synthesis transform: a smaller learned stand-in for g_s.       */
/*                                                                          */
/* The paper points to optimisations of the neural model itself as the     */
/* complement of its system architecture (Sections I and VI).  This net     */
/* maps y_hat (M channels) to the image with three transposed convolutions */
/* of F hidden channels: T(M->F, 5x5, stride 2, pad 2, output pad 1), ReLU, */
/* T(F->F, same), ReLU, T(F->3, 8x8, stride 4, pad 2): 16x upsampling, the  */
/* same as g_s.  It is trained on the GPU, by these entry points, to match */
/* the full g_s (mean squared error, AdamW), and can replace g_s in the     */
/* codec's decoder (codec_load_distilled).                                  */
/*                                                                          */
/* Parameters are one float32 array in this order: t1.w [M][F][5][5],      */
/* t1.b [F], t2.w [F][F][5][5], t2.b [F], t3.w [F][3][8][8], t3.b [3]       */
/* (transposed-convolution weights are [C_in][C_out][k][k]).  The handle    */
/* keeps an FP32 master copy with the AdamW moments; forward passes use     */
/* FP32 or bf16 GEMM operands (precision), gradients are FP32.  All tensor  */
/* arguments are device pointers on the handle's device unless stated.      */
/* ------------------------------------------------------------------------ */
typedef struct lic_distill lic_distill_t;

typedef struct {
    uint32_t struct_size;      /* sizeof(lic_distill_config)                         */
    int32_t  M, F;             /* latent channels (192 or 320), hidden channels (64) */
    int32_t  precision;        /* forward GEMM operands: LIC_PREC_FP32 / _BF16;      */
                               /* training (grads / step) requires LIC_PREC_FP32     */
    int32_t  max_batch;        /* largest n of any call                              */
    int32_t  max_hy, max_wy;   /* largest latent grid (image = 16 hy x 16 wy)        */
    int32_t  train;            /* 1: allocate gradient and optimizer state           */
    double   lr, beta1, beta2, eps, weight_decay;   /* AdamW (update runs in FP32)   */
    int32_t  hip_device;
} lic_distill_config;

/* M 192, F 64, FP32, batch 32, 16 x 16 latents, training on, lr 1e-3,
 * betas (0.9, 0.999), eps 1e-8, weight decay 0.01, device 0. */
void   lic_distill_default_config(lic_distill_config* cfg);
/* Number of float32 parameters for (M, F). */
size_t lic_distill_param_count(int M, int F);
/* params: host array of lic_distill_param_count(M, F) floats (copied). */
int    lic_distill_create(const lic_distill_config* cfg, const float* params, size_t n_params,
                          lic_distill_t** out);
void   lic_distill_destroy(lic_distill_t* d);
const char* lic_distill_last_error(const lic_distill_t* d);
/* Forward pass of n latents.  sym: int8 symbols NHWC [n][hy][wy][M] with
 * y_hat = sym + mu[c] (mu: M floats on the device, NULL = 0).  pre: NULL or
 * the unclamped output NCHW [n][3][16 hy][16 wy]; x_hat: NULL or the image
 * clamped to [0, 1] and cropped to H x W (NCHW [n][3][H][W]).  Runs on the
 * handle's stream and waits for it. */
int lic_distill_forward(lic_distill_t* d, const int8_t* sym, const float* mu, int n, int hy, int wy,
                        float* pre, float* x_hat, int H, int W);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass as lic_distill_forward, with the two hidden activations in a
 * fixed workspace of 32 MiB that the library holds per device instead of the
 * handle's buffers.  The call allocates nothing (the first call on a device
 * looks the workspace up once).  Needs 80 * n * hy * wy * F bytes with FP32
 * operands, 40 * n * hy * wy * F with bf16 (plus up to 255 of alignment):
 * LIC_E_BUDGET beyond the 32 MiB (one 720p frame, hy 48 x wy 80, F 64,
 * fits in either precision).  Every
 * call on one device shares that workspace, so calls that overlap on one
 * GPU (several threads or handles) race; nothing in it needs to start at
 * zero.  Runs on the handle's stream and waits for it. */
int lic_distill_forward_noalloc(lic_distill_t* d, const int8_t* sym, const float* mu, int n, int hy, int wy,
                                float* pre, float* x_hat, int H, int W);
/* Loss (mean squared error of the unclamped output against target, NCHW
 * [n][3][16 hy][16 wy]) and its gradient w.r.t. every parameter, without an
 * update.  grads: host array of param_count floats, or NULL; loss: host. */
int lic_distill_grads(lic_distill_t* d, const int8_t* sym, const float* mu, const float* target, int n,
                      int hy, int wy, float* grads, float* loss);
/* One training step on a batch drawn from a device-resident data set of
 * pairs (sym_all [count][hy][wy][M], target_all [count][3][16 hy][16 wy]):
 * idx (host, n entries < count) selects the samples, which are gathered on
 * the device; then forward, loss, backward and one AdamW update.  The loss
 * of the step goes to loss_dev[0] (device float, may be NULL).  Does not
 * wait for the GPU. */
int lic_distill_step(lic_distill_t* d, const int8_t* sym_all, const float* mu, const float* target_all,
                     long count, const int32_t* idx, int n, int hy, int wy, float* loss_dev);
/* Waits for every step issued so far. */
int lic_distill_sync(lic_distill_t* d);
/* Host copies of the state: what 0 = parameters, 1 = first moments,
 * 2 = second moments, 3 = last gradients; each param_count floats. */
int lic_distill_get(lic_distill_t* d, int what, float* out, size_t n);
/* Replaces parameters (what 0) or moments (1, 2) from host memory. */
int lic_distill_set(lic_distill_t* d, int what, const float* in, size_t n);
/* AdamW step counter (for resuming from a checkpoint). */
int lic_distill_get_step(lic_distill_t* d, int64_t* t);
int lic_distill_set_step(lic_distill_t* d, int64_t t);

/* ------------------------------------------------------------------------ */
/* Host entropy primitives (no GPU needed).                                 */
/* ------------------------------------------------------------------------ */
/* Byte-wise rANS (32-bit state, L = 2^23, 16-bit frequencies).  sym holds
 * alphabet indices 0..128 (value + 64), tab the table of each symbol, freq
 * is [ntab][129].  Returns the stream length, or LIC_E_SMALLBUF. */
long lic_rans_encode(const uint8_t* sym, const uint8_t* tab, long n,
                     const uint32_t* freq, int ntab, uint8_t* out, size_t cap);
/* Returns LIC_OK, or LIC_E_CORRUPT if the stream is truncated or does not
 * end in the initial state with every byte consumed. */
int  lic_rans_decode(const uint8_t* in, size_t len, const uint8_t* tab, long n,
                     const uint32_t* freq, int ntab, uint8_t* sym);
/* Interleaved word-wise rANS: the faster entropy coding the paper points to
 * (Sections II and VII).  `lanes` = K coder states (2, 4, 8, 16 or 32) share
 * one stream; symbol i is coded by state i mod K, so K independent chains
 * run side by side in one thread.  States are 32 bits in [2^16, 2^32) and
 * exchange 16-bit words with the stream; frequencies as above.  Stream: the
 * K final states (u32 little-endian, state 0 first), then the words (u16
 * little-endian) in the reverse of the order the encoder pushed them.  At
 * most 2 n + 4 K bytes.  Returns the stream length, LIC_E_SMALLBUF, or
 * LIC_E_ARG (bad lanes, symbol or table). */
long lic_rans_ileave_encode(int lanes, const uint8_t* sym, const uint8_t* tab, long n,
                            const uint32_t* freq, int ntab, uint8_t* out, size_t cap);
/* LIC_OK, or LIC_E_CORRUPT if the stream is truncated or does not end with
 * every state back at 2^16 and every word read. */
int  lic_rans_ileave_decode(int lanes, const uint8_t* in, size_t len, const uint8_t* tab, long n,
                            const uint32_t* freq, int ntab, uint8_t* sym);
/* FNV-1a 32-bit hash (the model id carried in every bitstream). */
uint32_t lic_fnv1a(const void* data, size_t len);
/* Entropy tables a codec would build from this weight blob, computed on the
 * host without a GPU: which 0 = factorized [C][129], 1 = Gaussian [64][129].
 * The float32 channel offsets (medians of the factorized densities) go to mu
 * when mu != NULL.  Returns the number of uint32 written, or a negative
 * lic_status (LIC_E_SMALLBUF if freq or mu is too small). */
long lic_blob_tables(const void* blob, size_t len, int which, uint32_t* freq, size_t cap,
                     float* mu, size_t mu_cap);

#ifdef __cplusplus
}
#endif
#endif /* LIC_H */
