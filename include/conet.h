/* conet.h — C ABI of the CoNet-Rx receiver library for AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Sec. II, the problem statement after Eq. (1)): given the
 * received grid of all OFDM symbols and subcarriers of one slot, return a soft bit
 * (LLR) for every bit of every resource element (RE). The network is the
 * collaborative receiver of Sec. III: K branches (k = 0 is the main net, the others
 * are support nets) each read the whole grid through a 3x3 conv + ReLU input layer,
 * then L pre-activation residual blocks (Sec. II-A, Fig. 1; the main net's block
 * after a fusion is the modified block of Fig. 3, without its leading
 * normalisation); after block l, if bit l-1 of fuse_mask is set, the block outputs
 * of all branches are multiplied element-wise and normalised per RE over the C
 * channels (LayerNorm) before entering the main net (Sec. III, and its extension to
 * M support nets); a 1x1 conv with one filter per bit of the symbol gives the LLRs
 * (Sec. III, output layer).
 *
 * Conventions
 *   - Tensors are channels-last: x[b][t][f][c] with t the OFDM symbol (T <= 14) and f
 *     the subcarrier; RE index = (b*T + t)*F + f.
 *   - Input features (Sec. II-A: Re/Im of the received grid; here also of the LS
 *     channel estimate): C_in = 4*N_rx channels, antenna-major
 *     (Re y_n, Im y_n, Re H_n, Im H_n), FP32.
 *   - LLR output: llr[b][t][f][j], FP32, j < bits_per_symbol, LLR = ln P(b=1)/P(b=0).
 *   - Pointers named *_host are host memory; every other tensor pointer is DEVICE
 *     memory of the GPU that was current when the model was created.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream). Calls that take
 *     a stream only enqueue work; buffers must stay valid until that work completes.
 *   - Every call returns a conet_status and never throws or aborts. On failure,
 *     conet_last_error() returns a message for the calling thread.
 *   - A model is used from one stream at a time; calls on one model must not overlap.
 */
#ifndef CONET_H
#define CONET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CONET_OK = 0,
  CONET_EINVAL = 1,   /* bad argument (null pointer, unsupported configuration) */
  CONET_ESHAPE = 2,   /* tensor shape outside what the model was created for */
  CONET_ENOMEM = 3,   /* workspace too small */
  CONET_EDEVICE = 4,  /* a HIP call failed; the HIP error string is in conet_last_error() */
  CONET_EBUSY = 5,    /* serving queue full */
  CONET_ETIMEOUT = 6, /* serving wait timed out */
  CONET_ESTATE = 7    /* call out of order (e.g. backward without a saved forward) */
} conet_status;

typedef enum {
  CONET_FP32 = 0,     /* FP32 MFMA operands and activations */
  CONET_BF16 = 1,     /* BF16 operands and activations, FP32 accumulation and epilogues */
  CONET_FP8E4M3 = 2,  /* OCP e4m3 conv operands (per-output-channel filter scales, static
                         per-tensor activation scales), BF16 residual stream, FP32 accumulation */
  CONET_FP64 = 3      /* not accepted by conet_create: no FP64 build of the kernels */
} conet_dtype;

typedef struct {
  int32_t branches;        /* K, 1..8; branch 0 is the main net                           */
  int32_t blocks;          /* L >= 1 residual blocks per branch                           */
  int32_t channels;        /* C: 16, 32, 64 or 96                                          */
  int32_t in_channels;     /* C_in = 4 N_rx: 8, 16 or 32; 4 N_rx + 8 = 24 (BF16, FP32) with the
                              noise / interference variance channels                      */
  int32_t bits_per_symbol; /* m, head width, 1..8                                          */
  uint32_t fuse_mask;      /* bit l-1 => fusion + LayerNorm after block l                  */
  float ln_eps;            /* LayerNorm epsilon (1e-5)                                     */
  int32_t dtype;           /* conet_dtype                                                  */
  int32_t train;           /* 1 => FP32 master weights, gradients, Adam state, per-block saved
                              activations (FP32 or BF16; C in {16,32,64}, C_in in {16,32}, K <= 4) */
  int64_t max_res;         /* largest B*T*F one call may pass                              */
  int32_t fusion_op;       /* CONET_FUSE_PRODUCT (0): P = prod_k O[k] (Sec. III, Example I);
                              CONET_FUSE_SUM (1): P = sum_k O[k] (fusion by addition, Sec. III) */
  int32_t feedback;        /* 1 => Example II (Sec. III): after each fusion, support branch k
                              continues from O[k] + the main branch's fused activation. The
                              training calls support fusion_op = 0, feedback = 0 only          */
  int32_t norm;            /* normalisation after each fusion (Sec. III allows BN or LN):
                              CONET_NORM_LN (0): per-RE LayerNorm over C, gamma/beta affine;
                              CONET_NORM_BN (1): BatchNorm, gamma (P - mean) / sqrt(var +
                              ln_eps) + beta per channel; the blob then ends with the running
                              statistics mean_l, var_l (C each) for l = 1..L. With train = 0
                              mean/var are those running statistics. With train = 1 (C in
                              {32, 64}) every forward normalises by the batch's own statistics
                              (over all B T F REs of the call, variance biased), conet_backward
                              differentiates through them, and each save_for_backward forward
                              moves the running statistics by CONET_BN_MOMENTUM towards the
                              batch's (variance unbiased, n/(n-1)); conet_get_weights returns
                              them for an inference model                                      */
  int32_t support_blocks;  /* blocks of every support branch, 1..L; 0 => L. Sec. III lets the
                              support net be shallower than the main net: after block
                              support_blocks the main branch continues alone, so fuse_mask may
                              only hold bits 0 .. support_blocks - 1. Inference only          */
  int32_t block_type;      /* CONET_BLOCK_STANDARD (0): 3x3 convs; CONET_BLOCK_SEPARABLE (1):
                              each block conv is a depthwise 3x3 filter followed by a 1x1 conv
                              (Sec. II-A). Separable: FP32 or BF16, C in {32, 64}, inference  */
} conet_config;

/* CONET_FUSE_CONCAT: P = Wc_l [O[0]; O[1]; ...; O[K-1]] + bc_l, the K outputs side by side
 * (K C channels) projected back to C by a 1x1 conv per block (Sec. III names concatenation
 * as a fusion operation), then the normalisation. FP32 or BF16, C in {32, 64}, K <= 4,
 * inference only. */
enum { CONET_FUSE_PRODUCT = 0, CONET_FUSE_SUM = 1, CONET_FUSE_CONCAT = 2 };
enum { CONET_NORM_LN = 0, CONET_NORM_BN = 1 };
/* running <- (1 - momentum) running + momentum batch, per BatchNorm training forward */
#define CONET_BN_MOMENTUM 0.1f
enum { CONET_BLOCK_STANDARD = 0, CONET_BLOCK_SEPARABLE = 1 };

typedef struct conet_model conet_model;

/* Number of FP32 values in the packed parameter blob. Blob order (all FP32):
 *   for k in 0..K-1: W_in[C][C_in][3][3], b_in[C],
 *                    for l in 1..L_k: s0[C], o0[C], W1[C][C][3][3], b1[C], s1[C], o1[C],
 *                                     W2[C][C][3][3], b2[C]
 *   for l in 1..L: gamma[C], beta[C]
 *   W_h[m][C], b_h[m]
 *   [CONET_FUSE_CONCAT: for l in 1..L: Wc[C][K C], bc[C]]
 *   [CONET_NORM_BN: for l in 1..L: mean[C], var[C]]
 * L_0 = L and L_k = support_blocks (k >= 1). Separable blocks hold D1[C][3][3], P1[C][C]
 * in place of W1 and D2[C][3][3], P2[C][C] in place of W2 (depthwise filter, then the 1x1
 * conv; out(t,f,c) of the depthwise filter reads in(t+dt, f+df, c) with D[c][dt+1][df+1]).
 * Filters are indexed [out][in][dt+1][df+1] and correlate: out(t,f) reads in(t+dt, f+df).
 * s0/o0 and s1/o1 are the per-channel affines in front of the block's ReLUs (inference
 * form of its normalisations); s0/o0 are ignored in a main-net block after a fusion.
 * Returns 0 for an invalid configuration. */
size_t conet_weight_count(const conet_config* cfg);

/* Device bytes the caller must provide to conet_create (0 for an invalid config). */
size_t conet_workspace_bytes(const conet_config* cfg);

/* Build a model: validates cfg, packs the blob into the kernels' fragment layout and
 * copies it into `workspace` (device memory, >= conet_workspace_bytes(cfg), 256-byte
 * aligned, owned by the caller and kept alive until conet_destroy). Synchronous.
 * Errors: EINVAL (config, null pointers, n_weights mismatch), ENOMEM (workspace too
 * small), EDEVICE. */
conet_status conet_create(const conet_config* cfg, const float* weights_host, size_t n_weights,
                          void* workspace, size_t workspace_bytes, conet_model** out);

/* FP8 only: set the static activation scales s_a (one per conv input operand,
 * n = 1 + 2*K*L: index 0 the input layer, then 1 + 2*(k*L + l-1) + {0: first conv of
 * block l of branch k, 1: its second conv}). Operands are quantised as e4m3(a / s_a).
 * Errors: EINVAL (wrong n, non-positive scale, not an FP8 model). */
conet_status conet_set_act_scales(conet_model* model, const float* scales_host, size_t n);

/* FP8 only: derive the activation scales from a calibration batch x (device, FP32,
 * [B][T][F][C_in]): each conv's scale is max|operand| / 448 over the batch, taken in
 * network order on the quantised forward. Synchronises the stream. */
conet_status conet_calibrate(conet_model* model, const float* x, int32_t B, int32_t T, int32_t F, void* stream);

/* Copy the current activation scales to host (n = 1 + 2*K*L). */
conet_status conet_get_act_scales(conet_model* model, float* scales_host, size_t n);

/* Forward pass: x (device, FP32 [B][T][F][C_in]) -> llr (device, FP32 [B][T][F][m]).
 * Every slot is padded with zeros at its own grid edges (no mixing between slots).
 * B == 0 is a no-op. With save_for_backward = 1 (train models only) every block's
 * input, middle activation and pre-fusion main output are kept for conet_backward, and
 * x must stay valid until then. Errors: EINVAL (null pointers), ESHAPE (T > 14, T < 1,
 * F < 1, B*T*F > max_res), ESTATE (save on an inference model), EDEVICE. */
conet_status conet_forward(conet_model* model, const float* x, int32_t B, int32_t T, int32_t F, float* llr,
                           int32_t save_for_backward, void* stream);

/* Forward pass over slots of different widths packed back to back: slot s has
 * T x F_host[s] REs starting at RE offset sum_{s'<s} T*F_host[s'] in x and llr.
 * Slots never share halos. Errors as conet_forward (sum T*F <= max_res). */
conet_status conet_forward_ragged(conet_model* model, const float* x, int32_t n_slots, int32_t T,
                                  const int32_t* F_host, float* llr, void* stream);

/* Bytes of the library's static device scratch array used by conet_forward_noalloc. */
#define CONET_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (HIP graph capture, serving loops that
 * forbid hipMalloc): conet_forward on a uniform batch, same arguments, layout and results
 * (bitwise), except that the forward's activation buffers (residual-stream ping-pong and
 * middle activations of every branch) come from a file-scope device array of
 * CONET_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load on that GPU until the
 * process ends, instead of the model's workspace. The call allocates nothing and enqueues
 * no memset. Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (any model, any stream) race and must be serialised by the caller. Inference only (no
 * save_for_backward). Errors: as conet_forward, plus ESHAPE when B*T*F exceeds
 * conet_forward_noalloc_capacity(model), EDEVICE when the current device is not the
 * model's, EINVAL for a BatchNorm model created with train = 1 (its batch statistics live
 * in the model's workspace). */
conet_status conet_forward_noalloc(conet_model* model, const float* x, int32_t B, int32_t T, int32_t F, float* llr,
                                   void* stream);

/* Largest B*T*F conet_forward_noalloc accepts for this model (its activation buffers
 * must fit the static array: at K = 3, C = 64 in BF16 about 58 K REs). 0 for a null model. */
int64_t conet_forward_noalloc_capacity(const conet_model* model);

/* conet_forward on a uniform batch with a HIP event recorded on `stream` before every
 * stage and after the last: stage_ms_host[i] (n_stages = 1 + 3L entries) gets the elapsed
 * time of stage i: the input layer, then per block (a) its first conv over all branches,
 * (b) the second conv of the support branches (with fusion) or of all branches (without),
 * (c) the second conv of the main branch with the fusion epilogue, LayerNorm and, after
 * the last block, the LLR head (0 without fusion).
 * When the model runs blocks as fused launches (conet_block_tile_width > 0), stage (a)
 * holds a block without fusion after it (both convs of every branch); (b) the support
 * branches of a fused block, in one launch with the previous block's main branch when that
 * is deferred to it (no Example II feedback); (c) a main branch launched alone (the last
 * block's, or one that could not be paired); unused entries are ~0.
 * stage_units_host (nullable, n_stages entries) receives per stage the conv-branch units it
 * ran: one conv of one branch over the whole batch (a fused block of one branch counts 2;
 * stage 0 counts the input conv of each branch), for per-stage FLOP accounting.
 * Synchronises on the last event. Errors as conet_forward. */
conet_status conet_forward_profiled(conet_model* model, const float* x, int32_t B, int32_t T, int32_t F, float* llr,
                                    float* stage_ms_host, int32_t* stage_units_host, int32_t n_stages, void* stream);

/* The network's input from the received grid (Sec. II, Eq. (1); Sec. II-A): least-squares
 * channel estimates at the fixed pilots (symbols 2 and 11, even subcarriers, value
 * (1+j)/sqrt(2)), interpolated linearly — odd subcarriers of a pilot symbol take the mean of
 * their even neighbours (a last odd one copies its left neighbour), and every symbol lies on
 * the line through symbols 2 and 11 — then laid out as the features conet_forward reads.
 * y: device FP32 [B][T][F][n_rx][2] (Re, Im); x_out: device FP32 [B][T][F][C_in] with
 * channels 4n..4n+3 = (Re y_n, Im y_n, Re H_n, Im H_n) for n < n_rx and zeros for the
 * remaining C_in/4 - n_rx antennas. FP32 arithmetic; enqueued on `stream`, no allocation.
 * Errors: EINVAL (null buffers), ESHAPE (T outside 12..14, B or F < 1, 4 n_rx > C_in, C_in not
 * a multiple of 4). */
conet_status conet_featurise(const float* y, int32_t B, int32_t T, int32_t F, int32_t n_rx, int32_t C_in,
                             float* x_out, void* stream);

/* Forward pass from the received grid: y (device, FP32 [B][T][F][n_rx][2], Re/Im per
 * antenna, the layout conet_featurise reads) -> llr (device, FP32 [B][T][F][m]). The input
 * layer forms the features while it stages its tiles -- the steps of conet_featurise (LS at
 * the pilots, linear interpolation; Sec. I and II-A), bit-identical to them -- so the
 * features never go through HBM; channels 4 n_rx .. C_in - 1 are zero (no variance
 * channels: models that take them run conet_featurise_var, then conet_forward). Same
 * results as conet_featurise followed by conet_forward. Errors: EINVAL (null pointers),
 * ESHAPE (T < 12 or T > 14, F < 1, n_rx < 1, 4 n_rx > C_in, B*T*F > max_res), ESTATE
 * (FP8 model without activation scales), EDEVICE. */
conet_status conet_forward_grid(conet_model* model, const float* y, int32_t B, int32_t T, int32_t F, int32_t n_rx,
                                float* llr, void* stream);

/* ---------------------------------------------------------------- recorded forward
 * A forward of fixed shape and buffers recorded once as a HIP graph and replayed with one
 * launch: at a batch of one slot the device otherwise waits for the host between the
 * forward's dependent kernels. conet_graph_create records conet_forward(model, x, B, T, F,
 * llr) (uniform batch, no save) on a private stream without running it; each
 * conet_graph_launch on `stream` then computes llr from the current contents of x, exactly
 * as conet_forward would. x, llr and the model must outlive the graph; replays of one graph
 * (or of graphs of one model) must not overlap in time: they share the model's activation
 * buffers. Errors: EINVAL (null arguments), ESHAPE (as conet_forward), ESTATE (FP8 model
 * without activation scales), EDEVICE. */
typedef struct conet_graph conet_graph;
conet_status conet_graph_create(conet_model* model, const float* x, int32_t B, int32_t T, int32_t F, float* llr,
                                conet_graph** out);
conet_status conet_graph_launch(conet_graph* graph, void* stream);
conet_status conet_graph_destroy(conet_graph* graph);

/* conet_featurise plus the known noise and interference variances of each slot, which the
 * receiver's input also carries (Sec. II-A concatenates them with the received grid):
 * variances: device FP32 [B][2] = (sigma_n^2, sigma_i^2) per slot. Channels C_in - 8 ..
 * C_in - 1 of every RE are (sigma_n^2, sigma_i^2, 0, 0, 0, 0, 0, 0); the antenna groups fill
 * channels 0 .. C_in - 9 (zeros beyond n_rx). Errors as conet_featurise (ESHAPE when 4 n_rx >
 * C_in - 8), EINVAL for null variances. */
conet_status conet_featurise_var(const float* y, const float* variances, int32_t B, int32_t T, int32_t F,
                                 int32_t n_rx, int32_t C_in, float* x_out, void* stream);

/* ---------------------------------------------------------------- on-device slot generator
 * Training batches generated on the GPU (the step before the receiver's input, Sec. II, Eq.
 * (1)): uniform bits, square Gray QAM with the fixed pilots (symbols 2 and 11, even
 * subcarriers, (1 + j)/sqrt(2)), a Rayleigh tapped-delay-line channel (n_taps taps 200 ns
 * apart, exponential power delay profile with 300 ns decay, unit total power) whose taps vary
 * over the slot by Clarke's isotropic scattering at a Doppler f_D ~ U[0, max_doppler_hz]
 * (16 sinusoids per tap and antenna), and white Gaussian noise of variance 10^(-SNR/10),
 * SNR ~ U[snr_lo_db, snr_hi_db] per slot; 30 kHz subcarriers, 14 symbols per 0.5 ms. Random
 * numbers: Philox4x32-10 keyed by `seed`, counter (slot, stream, index, 0), so slot s is the
 * same in any batch. */
typedef struct {
  int32_t F;                /* subcarriers                                              */
  int32_t T;                /* OFDM symbols, 12..14                                     */
  int32_t n_rx;             /* receive antennas, 1..8                                   */
  int32_t bits_per_symbol;  /* m: 2, 4, 6 or 8                                           */
  int32_t n_taps;           /* 1..16                                                    */
  float max_doppler_hz;
  float snr_lo_db, snr_hi_db;
  uint64_t seed;
} conet_sim_config;

/* Slots first_slot .. first_slot + B - 1: y (device, FP32 [B][T][F][n_rx][2], the layout
 * conet_featurise and conet_forward_grid read), bits (device, uint8 [B][T][F][m], 0/1; pilot
 * REs carry bits that were not sent), noise_var (device, FP32 [B], nullable). Errors:
 * EINVAL (null pointers, parameters out of range), ESHAPE (B > 65535, T, F), EDEVICE. */
conet_status conet_simulate(const conet_sim_config* cfg, int64_t first_slot, int32_t B, float* y, uint8_t* bits,
                            float* noise_var, void* stream);

/* Subcarriers per tile of the fused residual-block kernel that forwards of this model use
 * on a batch that fills the GPU (both convs of a block in one launch, the hidden activation
 * kept on chip): BF16 with C in {16, 32, 64} on 16x16 MFMAs, BF16 and FP8 with C = 96 on
 * 32x32 MFMAs, K <= 4. Training models (train = 1, C <= 64) run their save_for_backward
 * forwards on the same fused kernels, which then also store each block's middle activation.
 * Batches too small to fill the GPU run on narrower tiles of the same kernels. 0 when every
 * block runs as two conv launches (FP32, other widths, K > 4); FP8 calibration always does.
 * Returns 0 for a null model. */
int32_t conet_block_tile_width(const conet_model* model);

/* Dense-MFMA throughput on the current device, for reading roofline fractions against an
 * attainable peak: every wave of a full-chip grid (16 waves per CU) issues `iters` rounds
 * of 8 independent 16x16 MFMAs with register operands (dtype CONET_BF16: 16x16x32 bf16,
 * CONET_FP8E4M3: 16x16x128 f8, CONET_FP32: 16x16x4 f32), once to warm up and once timed.
 * *tflops_host gets the dense TFLOP/s of the timed run and *clock_ghz_host the shader
 * clock measured over one wave's loop (0 if the device does not report its wall-clock
 * rate). Allocates and frees a small device buffer: not for use under graph capture.
 * Errors: EINVAL (dtype, iters outside 1..2^24, null outputs), EDEVICE. */
conet_status conet_mfma_peak(int32_t dtype, int32_t iters, double* tflops_host, double* clock_ghz_host, void* stream);

/* The sum of a[k] b[k] (k < K) as ONE matrix instruction of a kind the conv kernels use
 * computes it, for checking how the instructions accumulate (the parity tolerances model it):
 * dtype CONET_BF16 with shape 16: v_mfma_f32_16x16x32_bf16 (K = 32), shape 32:
 * v_mfma_f32_32x32x16_bf16 (K = 16); CONET_FP8E4M3 with shape 16: the 16x16x128 e4m3
 * instruction (K = 128), shape 32: the 32x32x64 one (K = 64), unit scales. a_host, b_host: K
 * operand codes (BF16 bit patterns as uint16, or e4m3fn bytes). Synchronous; allocates and
 * frees a small device buffer. Errors: EINVAL (dtype, shape, null pointers), EDEVICE. */
conet_status conet_mfma_dot(int32_t dtype, int32_t shape, const void* a_host, const void* b_host, float* out_host);

/* ---------------------------------------------------------------- training
 * Reverse mode of the forward above (hand-written): the head, the per-RE LayerNorm,
 * the product fusion (d O[k] = dP * prod_{j != k} O[j]), and per block the input
 * gradient through both convs (flipped, transposed filters on the same implicit-GEMM
 * core; in BF16 at C = 32 and 64 both convs of a block run in one launch that keeps the
 * gradient between them on chip) and the filter gradients (a reduction over REs, in two
 * deterministic stages). */

/* Gradient of sum(llr * dllr) w.r.t. every parameter, from the last forward with
 * save_for_backward = 1 (dllr: device FP32 [B][T][F][m] of that forward). Overwrites
 * the gradient buffer (conet_grads). Errors: ESTATE (no saved forward, or an Adam step
 * since), EDEVICE. */
conet_status conet_backward(conet_model* model, const float* dllr, void* stream);

/* Device views (model-owned, FP32, blob order) of the gradients and master weights. */
conet_status conet_grads(conet_model* model, float** grads_dev, size_t* n);
conet_status conet_master_weights(conet_model* model, float** weights_dev, size_t* n);

/* One Adam step on the FP32 master copy (bias-corrected, step count kept by the model),
 * then every filter pack and per-channel vector is regenerated from it. */
conet_status conet_adam_step(conet_model* model, float lr, float beta1, float beta2, float eps, void* stream);

/* Copy the weights to host (n = conet_weight_count): the master copy of a train model,
 * else the blob it was created from. Synchronises the device. */
conet_status conet_get_weights(conet_model* model, float* weights_host, size_t n);

/* Training checkpoint (train models): copy the FP32 master weights and both Adam moments
 * (each n = conet_weight_count values in blob order) and the number of Adam steps taken to
 * host memory. Synchronises the device. Errors: EINVAL (null pointers, wrong n), ESTATE (not a
 * train model), EDEVICE. */
conet_status conet_save_train_state(conet_model* model, float* master_host, float* m_host, float* v_host, size_t n,
                                     int32_t* adam_steps);

/* Resume training from conet_save_train_state of a model with the same configuration: load the
 * master weights, the Adam moments and the step count, and regenerate every filter pack and
 * per-channel vector from the master copy, so that the next forward, backward and Adam step
 * are exactly those the saved model would have run. Drops a saved forward. Synchronous.
 * Errors: EINVAL (null pointers, wrong n, negative step count), ESTATE (not a train model),
 * EDEVICE. */
conet_status conet_load_train_state(conet_model* model, const float* master_host, const float* m_host,
                                     const float* v_host, size_t n, int32_t adam_steps);

/* Bitwise BCE with logits over data REs: loss_dev (1 float) = mean over the B slots'
 * data REs (data_mask [T][F] nonzero; n_data_per_slot of them) and their m bits of
 * max(z,0) - z b + log(1 + e^-|z|); dllr = (sigmoid(z) - b) / count on data REs, 0 on
 * pilots. bits: device uint8 [B][T][F][m]. */
conet_status conet_bce(conet_model* model, const float* llr, const uint8_t* bits, const uint8_t* data_mask, int32_t B,
                       int32_t T, int32_t F, int64_t n_data_per_slot, float* dllr, float* loss_dev, void* stream);

/* ---------------------------------------------------------------- serving
 * Continuous batching of slot requests (one TTI each). Each of the server's lanes (one HIP
 * stream + its own activation buffers) has a thread that forms a ragged batch whenever the
 * lane is free, taking queued requests in arrival order while their REs fit the lane
 * (admission by memory); batches on different lanes overlap on the device.
 * A request's LLRs do not depend on the other requests it is batched with. */
typedef struct conet_server conet_server;

typedef struct {
  int32_t n_prb;            /* PRBs: F = 12 * n_prb subcarriers                              */
  int32_t n_rx;             /* receive antennas; features have 4*n_rx channels (<= C_in), the
                               missing antennas are zero-padded                               */
  int32_t bits_per_symbol;  /* m of the request (<= the model's head width): LLR channels 0..m-1 */
  int32_t T;                /* OFDM symbols (1..14; all requests of a server share T)        */
  const float* x_host;      /* host FP32 input, read when the request is batched: features
                               [T][F][4*n_rx] (input = CONET_INPUT_FEATURES), or the received
                               grid [T][F][n_rx][2] (Re, Im; input = CONET_INPUT_GRID).
                               Page-locked memory (hipHostMalloc) is read by DMA with no host
                               copy, for grids and for features with all C_in channels; other
                               inputs are packed into the server's pinned staging first     */
  float* llr_host;          /* host [T][F][m] FP32 output; written before conet_serve_wait
                               returns. Page-locked memory is written by DMA; other buffers
                               receive a host copy from the server's pinned staging         */
  uint64_t tag;             /* caller's value, unused by the library                        */
  int32_t input;            /* CONET_INPUT_FEATURES (0) or CONET_INPUT_GRID (1): the server forms
                               the features on the GPU with conet_featurise (pilots on symbols
                               2 and 11, so T >= 12); half (4 rx) or a quarter (2 rx) of the
                               bytes to pack and copy                                         */
} conet_request;

enum { CONET_INPUT_FEATURES = 0, CONET_INPUT_GRID = 1 };

typedef struct {
  double p50_us, p99_us, mean_us, max_us;  /* latency: submit -> LLRs in llr_host           */
  double res_per_s;                        /* completed REs / (last completion - first submit) */
  double mean_batch_requests;
  uint64_t completed, rejected, batches;
  int64_t lane_res;                        /* REs one lane admits                          */
  /* where the mean latency goes, per completed request: waiting in the queue; forming its
   * batch (feature packing, enqueueing copies and kernels); enqueued -> the batch's
   * completion seen on the host (H2D, forward, D2H, plus the wait's wake-up); copying
   * the LLRs from pinned staging to the callers' buffers that are not page-locked */
  double mean_queue_us, mean_prep_us, mean_device_us, mean_scatter_us;
  /* GPU-timed parts of the device phase (stream events): the input copies, the forward
   * (with featurisation and the packing of narrower LLRs), the LLR copies of the batch */
  double mean_h2d_us, mean_forward_us, mean_d2h_us;
  /* completed requests whose input / LLRs went by DMA straight from / to the caller's
   * page-locked buffer */
  uint64_t direct_inputs, direct_outputs;
  /* the same four phases for the slowest completed request (its latency is max_us) */
  double slowest_queue_us, slowest_prep_us, slowest_device_us, slowest_scatter_us;
} conet_serve_stats;

/* Start a server on `model` (which must outlive it): n_streams lanes of up to
 * max_batch_res REs each, reduced until all lanes' device buffers fit mem_budget_bytes;
 * at most max_queue requests wait. Allocates its device and pinned host buffers here,
 * once. Errors: EINVAL (also for a BatchNorm model created with train = 1: batch
 * statistics would make a request's LLRs depend on the others in its batch), ENOMEM
 * (budget too small for one RE per lane), ESTATE (FP8 model without scales), EDEVICE. */
conet_status conet_serve_create(conet_model* model, size_t mem_budget_bytes, int32_t n_streams, int32_t max_batch_res,
                                int32_t max_queue, conet_server** out);

/* Queue one request (non-blocking). The request's buffers belong to the library until
 * conet_serve_wait returns for the ticket. Errors: EINVAL, ESHAPE (does not fit the
 * model or a lane), EBUSY (queue full: retry later). */
conet_status conet_serve_submit(conet_server* server, const conet_request* request, uint64_t* ticket);

/* Wait for a ticket (timeout_us < 0: no limit). On success *latency_us (nullable) is the
 * time from submit to the LLRs being in llr_host. Errors: ETIMEOUT (still pending; wait
 * again), EINVAL (unknown or already-collected ticket), EDEVICE. */
conet_status conet_serve_wait(conet_server* server, uint64_t ticket, int64_t timeout_us, double* latency_us);

/* Latency percentiles and throughput since creation or the last reset. */
conet_status conet_serve_get_stats(conet_server* server, conet_serve_stats* stats);
conet_status conet_serve_reset_stats(conet_server* server);

/* Stop (paused != 0) or resume forming new batches; batches in flight complete and
 * submissions are still queued (up to max_queue) while paused. */
conet_status conet_serve_pause(conet_server* server, int32_t paused);

/* Drain queued and in-flight requests (resuming a paused server), stop the threads,
 * free the server's buffers. */
conet_status conet_serve_destroy(conet_server* server);

/* Release the model (the caller frees the workspace afterwards). Synchronous. */
conet_status conet_destroy(conet_model* model);

/* Message of the last failed call on this thread ("" if none). */
const char* conet_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CONET_H */
