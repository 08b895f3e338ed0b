/*
 * gsc.h -- C ABI of the MI355X (gfx950) Gaussian-frame codec: the per-frame hot path of GS-NFS
 * (arXiv 2606.05650) -- positions as octree occupancy bytes, attributes as quantized RAHT
 * coefficients.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* are device pointers (HIP device memory of the current device); all
 *   others are host pointers. The caller owns every buffer; the library never allocates or
 *   frees memory, and never synchronizes the stream.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream). Every call only
 *   enqueues work on that stream and returns; results are valid once the stream has been
 *   synchronized.
 * - Concurrency: calls on one device must not run at the same time on different streams. The
 *   transform launches that run the upper RAHT levels (the forward, and the inverse of the upper
 *   levels) keep all their workgroups resident and order the levels by waiting on one another;
 *   a concurrent call's kernels can take the slots they wait for, and the call then fails with
 *   GSC_ERR_INTERNAL after a bounded wait. Serialize calls on a
 *   device (one stream, or events between streams); frames coded together belong in one batch
 *   call. The host side is thread-safe: the only process-wide state (the sort tuning table and
 *   per-device launch limits) is guarded.
 * - Argument errors are returned synchronously as a gsc_status and nothing is enqueued. Device
 *   buffers of one call (or of all frames of a batch) must not overlap where either is written:
 *   every entry point compares the byte ranges it will touch ([ptr, ptr + bytes) of each input,
 *   output, workspace and info array, sized from the arguments) and returns GSC_ERR_INVALID_ARG
 *   for an overlap. Read-only inputs may overlap each other.
 * - Errors found on the device (a corrupt stream, a capacity overflow) are written as a
 *   gsc_status code to the device info word of the call (see gsc_info) and every later kernel
 *   of the same call returns without writing outputs.
 * - Integers in device buffers are little-endian. Float attributes are IEEE binary32.
 *
 * Octree depth J is 1..21 (Morton codes are 3J <= 63 bits, Sec. 2.2), channels C are 1..64.
 */
#ifndef GSC_H
#define GSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSC_MAX_DEPTH 21
#define GSC_MAX_CHANNELS 64
#define GSC_MAX_BATCH 64
#define GSC_HEADER_BYTES 1024u
#define GSC_MAGIC 0x31435347u /* "GSC1" */
#define GSC_VERSION 1u

typedef enum gsc_status {
    GSC_OK = 0,
    GSC_ERR_INVALID_ARG = 1,    /* null pointer, negative size, bad step or tau          */
    GSC_ERR_DEPTH = 2,          /* J outside 1..21 or C outside 1..64                    */
    GSC_ERR_WORKSPACE = 3,      /* workspace smaller than gsc_workspace_size()           */
    GSC_ERR_CAPACITY = 4,       /* output buffer smaller than required                   */
    GSC_ERR_CORRUPT_STREAM = 5, /* header or occupancy bytes inconsistent (device-side)  */
    GSC_ERR_HIP = 6,            /* a HIP launch failed                                   */
    GSC_ERR_INTERNAL = 7,       /* a device-side invariant failed (a bug; please report) */
    GSC_ERR_SCRATCH = 8         /* frame needs more than GSC_STATIC_SCRATCH_BYTES of
                                   workspace (gsc_encode_frame_noalloc only)             */
} gsc_status;

/* Coding parameters of one frame.
 * quant_step[c] > 0 is the uniform quantization step of channel c, used for every RAHT
 * coefficient of that channel (Sec. 3.4); q = sgn(y) floor(|y|/step + tau), y^ = q * step.
 * tau in [0, 1): 0.5 rounds half away from zero; smaller values widen the dead zone.
 * bbox_mode 0 voxelizes inside the cube bounding the frame (per-axis minimum, cell =
 * largest extent / 2^J, Sec. 2.1); bbox_mode 1 uses bbox_min and cell as given (points
 * outside the box are clamped into it), which keeps the grid fixed across a sequence. */
typedef struct gsc_params {
    int32_t J;
    int32_t C;
    float quant_step[GSC_MAX_CHANNELS];
    float tau;
    int32_t bbox_mode;
    double bbox_min[3];
    double cell;
    uint32_t flags;          /* GSC_FLAG_* below; 0 = defaults */
    uint32_t reserved;       /* must be 0 */
} gsc_params;

/* flags: GSC_FLAG_FP64_WEIGHTS computes every butterfly's rotation (a, b) = (sqrt(w0/(w0+w1)),
 * sqrt(w1/(w0+w1))) of Eq. 1 in FP64 and rounds it once to FP32 (default: FP32 division and
 * square root, within about one FP32 ulp of the same value; the butterflies themselves are FP32
 * either way). The flag is recorded in the stream header and the decoder follows it. Weights
 * are integer leaf counts, exact in FP32 up to 2^24 voxels. */
#define GSC_FLAG_FP64_WEIGHTS 0x1u
#define GSC_FLAGS_KNOWN 0x1u

/* Layout of the encoded stream (the first GSC_HEADER_BYTES of every stream).
 * Byte layout: [header][occupancy bytes: levels 0..J-1, each in Morton order, one byte per
 * internal node, bit i set <=> child (p << 3) + i occupied (Sec. 2.2, Alg. 1)][zero padding
 * to a multiple of 256][coefficients: int32, Nv rows x C channels, row-major; row 0 holds the
 * DC, row i > 0 the high-pass coefficient stored at voxel i (Sec. 3.1, Alg. 6)]. */
typedef struct gsc_header {
    uint32_t magic;          /* GSC_MAGIC                                      */
    uint32_t version;        /* GSC_VERSION                                    */
    uint32_t J, C;           /* octree depth and channel count                 */
    uint32_t n_in;           /* Gaussians in the encoded frame                 */
    uint32_t n_vox;          /* occupied voxels Nv = |L_J|                     */
    uint32_t level_sizes[22];/* |L_0| .. |L_J| (Alg. 1 step 3), rest zero      */
    uint32_t error;          /* 0, or the gsc_status the encoder failed with   */
    uint32_t flags;          /* gsc_params.flags of the encoder                */
    double bbox_min[3];      /* voxel grid origin                              */
    double cell;             /* voxel edge length                              */
    float quant_step[64];    /* per-channel steps, C used                      */
    float tau;
    uint32_t reserved1;
    uint64_t occ_offset;     /* = GSC_HEADER_BYTES                             */
    uint64_t occ_bytes;      /* sum of |L_d| for d < J                         */
    uint64_t coef_offset;    /* 256-byte aligned                               */
    uint64_t coef_bytes;     /* Nv * C * 4                                     */
    uint64_t total_bytes;    /* coef_offset + coef_bytes                       */
} gsc_header;

/* Device info words written by every call: [0] gsc_status of the device side (0 = ok),
 * [1] Nv, [2..3] stream bytes (encode) as uint64, [4] number of RAHT tiling levels used. */
#define GSC_INFO_WORDS 8

/* ------------------------------------------------------------------------------------------
 * Sizes.
 * gsc_workspace_size: device scratch bytes needed by one call on frames of at most n_max
 *   Gaussians (encode) or voxels (decode) at depth J with C channels. Returns GSC_OK.
 * gsc_stream_capacity: worst-case encoded stream bytes for such a frame (header + one byte
 *   per possible internal node + padding + n_max * C coefficients).
 * ---------------------------------------------------------------------------------------- */
gsc_status gsc_workspace_size(int64_t n_max, int32_t J, int32_t C, size_t *bytes);
gsc_status gsc_stream_capacity(int64_t n_max, int32_t J, int32_t C, size_t *bytes);

/* ------------------------------------------------------------------------------------------
 * gsc_encode_frame -- encode one frame (Sec. 2.2 voxelization, octree construction and
 * bitstream generation, Alg. 1; Sec. 3.2-3.4 RAHT prelude, transform and quantization,
 * Alg. 4-6).
 *   d_pos    [n][3] float positions, d_attr [n][C] float attributes (row-major).
 *   d_stream output stream of stream_cap bytes (>= gsc_stream_capacity(n, J, C)).
 *   d_ws     workspace of ws_bytes (>= gsc_workspace_size(n, J, C)).
 *   d_info   device int32[GSC_INFO_WORDS] written with the device status and sizes.
 *   d_coef_f32 optional [n][C] float: the unquantized coefficients (rows 0..Nv-1), or NULL.
 *   d_leaf_codes optional [n] uint64: the sorted voxel Morton codes L_J, or NULL.
 *   d_perm optional [n] uint32: the stable sorted order of the Gaussians by Morton code
 *     (Alg. 1 step 1; equal codes keep their input order): d_perm[k] is the input row of the
 *     k-th Gaussian in sorted order, or NULL.
 *   d_voxel_of optional [n] uint32: the voxel (row of the decoded frame, 0..Nv-1) each input
 *     Gaussian was merged into, or NULL.
 * Positions must be finite. n may be 0 (an empty stream). Duplicates (Gaussians in one
 * voxel) are replaced by one voxel whose attributes are their mean (Sec. 2.1).
 * ---------------------------------------------------------------------------------------- */
gsc_status gsc_encode_frame(const float *d_pos, const float *d_attr, int64_t n,
                            const gsc_params *params, void *d_stream, size_t stream_cap,
                            void *d_ws, size_t ws_bytes, int32_t *d_info, float *d_coef_f32,
                            uint64_t *d_leaf_codes, uint32_t *d_perm, uint32_t *d_voxel_of,
                            void *stream);

/* ------------------------------------------------------------------------------------------
 * gsc_encode_frame_noalloc -- gsc_encode_frame without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). The workspace is a static device array of GSC_STATIC_SCRATCH_BYTES
 * that the library's code object holds on every device it runs on, from its load until the
 * process ends; its device address is looked up once per device (hipGetSymbolAddress, on the
 * first call made with that device current). The call allocates and frees nothing; the caller
 * still passes every input and output exactly as for gsc_encode_frame, and the outputs are
 * identical to that call's.
 *   Limit: frames whose gsc_workspace_size(n, J, C) exceeds GSC_STATIC_SCRATCH_BYTES return
 *   GSC_ERR_SCRATCH before anything is enqueued (about 530K Gaussians at J = 12, C = 56).
 *   Concurrency: every call on a device shares that device's one array, which keeps the last
 *   call's contents (the call clears what must start at zero itself). Calls whose work
 *   overlaps on one device race and corrupt each other's results: order them on one stream
 *   (or with events), and do not run this entry point at the same time as itself.
 * ---------------------------------------------------------------------------------------- */
#define GSC_STATIC_SCRATCH_BYTES (64u << 20)
gsc_status gsc_encode_frame_noalloc(const float *d_pos, const float *d_attr, int64_t n,
                                    const gsc_params *params, void *d_stream, size_t stream_cap,
                                    int32_t *d_info, float *d_coef_f32, uint64_t *d_leaf_codes,
                                    uint32_t *d_perm, uint32_t *d_voxel_of, void *stream);

/* ------------------------------------------------------------------------------------------
 * gsc_decode_frame -- decode one stream (Sec. 2.3 and Alg. 2-3 octree expansion and Morton
 * decode; Alg. 6 inverse RAHT after dequantization).
 *   d_stream, stream_bytes: an encoded stream on the device.
 *   J, C: the depth and channel count the caller expects; the header must agree.
 *   n_cap: capacity in voxels of the outputs (>= the stream's Nv).
 *   d_pos_out [n_cap][3] float voxel centres (bbox_min + (v + 1/2) * cell, in FP64 then
 *     rounded to float); d_vox_out optional [n_cap][3] uint32 voxel coordinates;
 *   d_attr_out [n_cap][C] float attributes; d_leaf_codes optional [n_cap] uint64.
 *   Rows are in Morton order; Nv is written to d_info[1].
 * A stream whose occupancy bytes do not reproduce its level sizes, or that has a zero byte,
 * is reported as GSC_ERR_CORRUPT_STREAM in d_info[0].
 * ---------------------------------------------------------------------------------------- */
gsc_status gsc_decode_frame(const void *d_stream, size_t stream_bytes, int32_t J, int32_t C,
                            int64_t n_cap, float *d_pos_out, uint32_t *d_vox_out,
                            float *d_attr_out, uint64_t *d_leaf_codes, void *d_ws,
                            size_t ws_bytes, int32_t *d_info, void *stream);

/* ------------------------------------------------------------------------------------------
 * gsc_encode_batch -- encode F frames (F <= GSC_MAX_BATCH) of uneven sizes with one launch
 * per pipeline stage for the whole batch (every kernel covers the tiles of all frames).
 * frames[f] gives frame f's inputs and outputs (host array of descriptors holding device
 * pointers); each frame needs its own workspace of gsc_workspace_size(n_f, J, C) bytes.
 * The results are identical, byte for byte, to F calls of gsc_encode_frame.
 * ---------------------------------------------------------------------------------------- */
typedef struct gsc_frame_desc {
    const float *d_pos;
    const float *d_attr;
    int64_t n;
    void *d_stream;
    size_t stream_cap;
    void *d_ws;
    size_t ws_bytes;
    int32_t *d_info;
} gsc_frame_desc;

gsc_status gsc_encode_batch(const gsc_frame_desc *frames, int32_t F, const gsc_params *params,
                            void *stream);

/* gsc_decode_batch -- decode F streams with one launch per stage (see gsc_encode_batch). */
typedef struct gsc_stream_desc {
    const void *d_stream;
    size_t stream_bytes;
    int64_t n_cap;
    float *d_pos_out;
    float *d_attr_out;
    void *d_ws;
    size_t ws_bytes;
    int32_t *d_info;
} gsc_stream_desc;

gsc_status gsc_decode_batch(const gsc_stream_desc *streams, int32_t F, int32_t J, int32_t C,
                            void *stream);

/* ------------------------------------------------------------------------------------------
 * Autotuning of the sort tiling (the Morton-code sort of Sec. 2.2 / Alg. 1 step 1).
 *
 * The radix sort of an encode call runs one of GSC_SORT_VARIANTS tilings (keys per workgroup
 * and look-back window width). Which one is fastest depends on the frame size: few large tiles
 * shorten the chain of tiles whose prefixes must be resolved, many small tiles fill more
 * compute units. The choice is kept in a process-wide table keyed by the depth J and the size
 * class ceil(log2(n_max)) of the largest frame of a call; untuned entries use the default
 * (variant 1, 2048-key tiles, for n_max <= 2^18; variant 0, 4096-key tiles, above). All variants
 * produce identical streams.
 *
 * gsc_autotune -- times every variant on the caller's batch (each timed as reps encodes of the
 *   whole batch after one warm-up, exactly as gsc_encode_batch runs it, on `stream`), stores
 *   the fastest in the table for this batch's key (the default instead, unless the fastest is
 *   at least 2 % faster than it) and returns it in *chosen (optional);
 *   times_ms (optional, GSC_SORT_VARIANTS floats) receives the mean time of each. Arguments
 *   and buffers as for gsc_encode_batch; the frames are encoded (the outputs of the last run
 *   remain). SYNCHRONOUS: it waits for the stream, so it must not be called while the stream
 *   is being captured into a graph. Allocates no device memory.
 * gsc_tune_set -- sets the entry for (J, size class of n) to `variant`, or clears it with -1.
 * gsc_tune_get -- the variant an encode call whose largest frame has n entries would use.
 * ---------------------------------------------------------------------------------------- */
#define GSC_SORT_VARIANTS 4
gsc_status gsc_autotune(const gsc_frame_desc *frames, int32_t F, const gsc_params *params,
                        int32_t reps, int32_t *chosen, float *times_ms, void *stream);
gsc_status gsc_tune_set(int32_t J, int64_t n, int32_t variant);
gsc_status gsc_tune_get(int32_t J, int64_t n, int32_t *variant);

/* ------------------------------------------------------------------------------------------
 * gsc_raht_forward / gsc_raht_adjoint -- the orthonormal transform alone, on float
 * attributes of voxels already in Morton order (Eq. 1 and Alg. 4-6 on all 3J levels):
 *   Y = T A (forward) and A = T^T Y (adjoint, which is the inverse since T is orthonormal).
 *   d_codes [nv] sorted distinct Morton codes; d_in, d_out [nv][C] float (may not alias).
 * The adjoint is the backward pass of the forward transform as a differentiable operation.
 * ---------------------------------------------------------------------------------------- */
gsc_status gsc_raht_forward(const uint64_t *d_codes, int64_t nv, int32_t J, int32_t C,
                            const float *d_in, float *d_out, void *d_ws, size_t ws_bytes,
                            int32_t *d_info, void *stream);
gsc_status gsc_raht_adjoint(const uint64_t *d_codes, int64_t nv, int32_t J, int32_t C,
                            const float *d_in, float *d_out, void *d_ws, size_t ws_bytes,
                            int32_t *d_info, void *stream);

/* ------------------------------------------------------------------------------------------
 * Straight-through (STE) attribute coding: the codec as a differentiable layer. The paper's
 * coder (Sec. 3: RAHT of Eq. 1 / Alg. 6 and the uniform quantizer of Sec. 3.4) has a
 * piecewise-constant quantizer; the straight-through form passes gradients through it as if it
 * were the identity, so a rate-distortion loss of the decoded attributes can be backpropagated
 * to the Gaussian attributes.
 *
 * gsc_ste_forward -- gsc_encode_frame (same arguments, same stream written) plus, for the Nv
 *   occupied voxels in Morton order:
 *     d_aref [n][C] (optional)   a = voxel means of the input rows (the rows RAHT transforms)
 *     d_yhat [n][C]              yhat = q * step (the dequantized coefficients, Alg. 6 layout:
 *                                row 0 the DC, row i > 0 the high-pass stored at voxel i)
 *     d_ahat [n][C]              ahat = T^T yhat (the attributes the decoder reconstructs)
 *   Rows Nv..n-1 are not written; Nv is d_info[1] after the call completes. d_yhat, d_ahat and
 *   d_attr must not alias. The workspace afterwards holds the transform schedule that
 *   gsc_ste_backward uses.
 *
 * gsc_ste_backward -- given dL/dyhat and dL/dahat ([Nv][C] float rows each, both required;
 *   pass zeros for a term the loss does not use), writes dL/dattr [n][C] for every input row:
 *     g_vox = dL/dahat + T^T dL/dyhat,  dL/dattr[i] = g_vox[voxel of i] / (Gaussians in it).
 *   This is T^T (T dL/dahat + dL/dyhat) with T^T T = I (T is orthonormal), the straight-through
 *   gradient (dyhat/dy taken as the identity) chained through the voxel mean. d_ws must be the
 *   workspace of a gsc_ste_forward call with the same n, J and C, not used by any other call
 *   since; otherwise d_info[0] reports GSC_ERR_INVALID_ARG. It may be called several times
 *   for the same forward. d_grad_attr must not alias the gradient inputs.
 * ---------------------------------------------------------------------------------------- */
gsc_status gsc_ste_forward(const float *d_pos, const float *d_attr, int64_t n,
                           const gsc_params *params, void *d_stream, size_t stream_cap, void *d_ws,
                           size_t ws_bytes, int32_t *d_info, float *d_yhat, float *d_ahat,
                           float *d_aref, uint64_t *d_leaf_codes, void *stream);
gsc_status gsc_ste_backward(int64_t n, int32_t J, int32_t C, const float *d_grad_yhat,
                            const float *d_grad_ahat, float *d_grad_attr, void *d_ws,
                            size_t ws_bytes, int32_t *d_info, void *stream);

/* ------------------------------------------------------------------------------------------
 * Block-parallel entropy coding of quantized coefficients (Sec. 3.4 "Quantization and Entropy
 * Coding": run-length / adaptive Golomb-Rice coding of independent blocks of consecutive
 * coefficients of one channel, coded in parallel).
 *   Input/output coefficients: [nv][C] int32, row-major (the coefficient section of an encoded
 *   stream is such a matrix: row 0 the DC, row i the high-pass stored at voxel i).
 *   Blocks: channel c's nv values, in row order, cut into blocks of B values (the last one
 *   shorter); block b = j * C + c holds rows j*B .. j*B + B - 1 of channel c, coded from a fresh
 *   coder state into a whole number of 32-bit words (bits from the most significant down).
 *   Coder (the paper names the method, not its parameters): adaptive run mode and Golomb-Rice
 *   parameters held with 3 fractional bits (both start at 8, kept in 0..80); run mode sends a 0
 *   bit per 2^k zeros (kp += 4), a 1 and the remaining count in k bits, then the sign and the
 *   Golomb-Rice code of |v| - 1 of the value that ends the run (kp -= 6); otherwise each value
 *   is sent as the Golomb-Rice code of 2v or -2v - 1 (kp += 3 after a zero, -= 3 otherwise).
 *   The Golomb-Rice code of u is u >> kr ones, a 0 and the kr low bits, or, when u >> kr >= 24,
 *   24 ones and u in 32 bits; krp -= 2 when u >> kr = 0 and += u >> kr when it is above 1.
 *   Stream: gsc_rlgr_header, then the blocks' first words uint32[nblocks + 1] (the last entry
 *   is total_words), then the total_words code words. Little-endian.
 * gsc_rlgr_capacity: worst-case stream bytes for nv x C values (68 bits per value plus a word
 *   per block, the header and the table). gsc_rlgr_workspace_size: device scratch bytes.
 * gsc_rlgr_encode: d_q [nv][C] -> d_out (out_cap bytes). d_info[0] device status (
 *   GSC_ERR_CAPACITY if the code does not fit out_cap), d_info[2..3] the stream bytes (uint64).
 * gsc_rlgr_decode: d_in (in_bytes) -> d_q [nv][C]; nv, C and B must match the header;
 *   GSC_ERR_CORRUPT_STREAM in d_info[0] for a header or a block that does not decode to exactly
 *   its values within its words (the rows of such a block are then unspecified).
 * B is 1 .. 65536; C 1 .. 64; nv < 2^30.
 * ---------------------------------------------------------------------------------------- */
#define GSC_RLGR_MAGIC 0x31474C52u /* "RLG1" */
typedef struct gsc_rlgr_header {
    uint32_t magic;          /* GSC_RLGR_MAGIC                     */
    uint32_t version;        /* GSC_VERSION                        */
    uint32_t nv, C, B;       /* rows, channels, block length       */
    uint32_t nblocks;        /* C * ceil(nv / B)                   */
    uint32_t total_words;    /* code words after the table         */
    uint32_t reserved;
} gsc_rlgr_header;

gsc_status gsc_rlgr_capacity(int64_t nv, int32_t C, int32_t B, size_t *bytes);
gsc_status gsc_rlgr_workspace_size(int64_t nv, int32_t B, size_t *bytes);
gsc_status gsc_rlgr_encode(const int32_t *d_q, int64_t nv, int32_t C, int32_t B, void *d_out,
                           size_t out_cap, void *d_ws, size_t ws_bytes, int32_t *d_info,
                           void *stream);
gsc_status gsc_rlgr_decode(const void *d_in, size_t in_bytes, int64_t nv, int32_t C, int32_t B,
                           int32_t *d_q, void *d_ws, size_t ws_bytes, int32_t *d_info,
                           void *stream);

/* ------------------------------------------------------------------------------------------
 * Entropy coding of the occupancy bytes (an own range-ANS coder in place of the closed ANS
 * library the paper uses for the geometry, Sec. 2.2 and Sec. 5). Any byte string; the codec's
 * occupancy section is bytes [occ_offset, occ_offset + occ_bytes) of an encoded stream.
 *   Model: one static table per stream over the 256 byte values with frequencies out of 4096:
 *   f_s = 1 + floor(c_s (4096 - P) / T) for a byte present c_s times among the T input bytes (P
 *   distinct bytes), the remainder to the most frequent byte (the smallest on a tie).
 *   Coder: 32-bit rANS with byte renormalisation (state in [2^23, 2^31)); the input is cut into
 *   chunks of K bytes (the last one shorter), each coded on its own from the state 2^23 with its
 *   symbols taken last to first and stored in reverse emission order (its final state first,
 *   most significant byte first), so a decoder reads each chunk forward; it accepts a chunk
 *   whose first state is at least 2^23 (an encoder's always is) and that ends in the state 2^23
 *   with every byte of the chunk consumed.
 *   Stream: gsc_rans_header, the table uint16[256], the chunks' first bytes uint32[nchunks + 1]
 *   (counted from the data; the last entry is `total`), then the data. Little-endian.
 * gsc_rans_capacity / gsc_rans_workspace_size: worst-case stream bytes (2 bytes per input byte
 *   and 4 per chunk, plus the header, table and offsets) and device scratch bytes.
 * gsc_rans_encode: d_in (n bytes) -> d_out (out_cap bytes); d_info[0] the device status
 *   (GSC_ERR_CAPACITY if the code does not fit), d_info[2..3] the stream bytes (uint64).
 * gsc_rans_decode: d_in (in_bytes) -> d_out (n bytes); n and K must match the header;
 *   GSC_ERR_CORRUPT_STREAM in d_info[0] for a header, table or chunk that does not decode as
 *   above (the bytes of such a chunk are then unspecified). d_ws: 8 bytes.
 * K is 1 .. 2^20; n < 2^31. Inputs and outputs must not overlap. The stream (d_out of the
 * encoder, d_in of the decoder) and d_ws must be 8-byte aligned, d_info 4-byte aligned
 * (GSC_ERR_INVALID_ARG otherwise); the raw bytes (the encoder's d_in, the decoder's d_out) may
 * start anywhere. The kernels read only whole aligned words that hold at least one byte of
 * their buffer, and read the bytes of a word that reaches outside it one by one.
 * ---------------------------------------------------------------------------------------- */
#define GSC_RANS_MAGIC 0x314E4152u /* "RAN1" */
typedef struct gsc_rans_header {
    uint32_t magic;          /* GSC_RANS_MAGIC                      */
    uint32_t version;        /* GSC_VERSION                         */
    uint64_t n;              /* input bytes                         */
    uint32_t K;              /* chunk length                        */
    uint32_t nchunks;        /* ceil(n / K)                         */
    uint32_t total;          /* data bytes after the offsets        */
    uint32_t reserved;
} gsc_rans_header;

gsc_status gsc_rans_capacity(int64_t n, int32_t K, size_t *bytes);
gsc_status gsc_rans_workspace_size(int64_t n, int32_t K, size_t *bytes);
gsc_status gsc_rans_encode(const void *d_in, int64_t n, int32_t K, void *d_out, size_t out_cap,
                           void *d_ws, size_t ws_bytes, int32_t *d_info, void *stream);
gsc_status gsc_rans_decode(const void *d_in, size_t in_bytes, int64_t n, int32_t K, void *d_out,
                           void *d_ws, size_t ws_bytes, int32_t *d_info, void *stream);

/* ------------------------------------------------------------------------------------------
 * Colour decorrelation before the transform (Sec. 4 "Improving Compression"): every SH
 * function's RGB triple goes to YUV, and each YUV channel gets its own per-frame Karhunen-Loeve
 * transform (KLT) over its 15 AC SH coefficients; the DC coefficients get the YUV step only.
 * A caller runs gsc_color_forward on the attribute rows before gsc_encode_frame and
 * gsc_color_inverse on the decoded rows, keeping the frame's three KLT matrices (2700 bytes) as
 * side information.
 *   Layout: [n][C] float32 rows; the 48 SH channels start at column sh0 (sh0 + 48 <= C): the DC
 *   of R, G, B, then the 15 AC functions of R, of G and of B (the storage order of degree-3
 *   Gaussian splats). The output keeps that layout with Y, U, V in place of R, G, B and KLT
 *   coefficient j in place of function j; columns outside [sh0, sh0 + 48) are copied.
 *   YUV (the paper gives no coefficients): the BT.601 definition, Kr = 0.299, Kb = 0.114,
 *   Umax = 0.436, Vmax = 0.615: Y = Kr R + (1 - Kr - Kb) G + Kb B, U = Umax (B - Y) / (1 - Kb),
 *   V = Vmax (R - Y) / (1 - Kr).
 *   KLT of channel c: the eigenvectors of the covariance (about the mean, over the n rows) of
 *   its 15 AC values, in decreasing eigenvalue order, each with its largest-magnitude component
 *   positive; d_klt[c][i][j] is component i of vector j; coefficients a = E^T x, inverse
 *   x = E a; with fewer than two rows every E is the identity.
 * gsc_color_workspace_size: device scratch bytes for n rows.
 * gsc_color_forward: d_attr -> d_out, d_klt float[3][15][15]; d_eig (double[3][15], may be
 *   NULL) the eigenvalues; d_info[0] = 0, d_info[1] = n once done.
 * gsc_color_inverse: d_coef (forward's layout) and d_klt -> d_out (RGB rows).
 * Inputs and outputs must not overlap; n < 2^31; C <= 64.
 * ---------------------------------------------------------------------------------------- */
#define GSC_COLOR_SH_CHANNELS 48
#define GSC_COLOR_KLT_FLOATS (3 * 15 * 15)
gsc_status gsc_color_workspace_size(int64_t n, size_t *bytes);
gsc_status gsc_color_forward(const float *d_attr, int64_t n, int32_t C, int32_t sh0, float *d_out,
                             float *d_klt, double *d_eig, void *d_ws, size_t ws_bytes,
                             int32_t *d_info, void *stream);
gsc_status gsc_color_inverse(const float *d_coef, int64_t n, int32_t C, int32_t sh0,
                             const float *d_klt, float *d_out, void *stream);

/* ------------------------------------------------------------------------------------------
 * Diagnostics: gsc_profile_events -- record caller-created HIP events around one stage of every
 * later call on the calling process (all threads share this setting). `events` holds n_pairs
 * (start, end) pairs of hipEvent_t (as void*); the i-th launch of the stage records pair
 * i % n_pairs on the call's stream, immediately before and after the stage. n_pairs = 0 (or
 * events = NULL) switches the stage off. Not for concurrent use with other profiling.
 * ---------------------------------------------------------------------------------------- */
typedef enum gsc_stage {
    GSC_STAGE_ENCODE = 0,      /* a whole gsc_encode_frame / gsc_encode_batch call           */
    GSC_STAGE_DECODE = 1,      /* a whole gsc_decode_frame / gsc_decode_batch call           */
    GSC_STAGE_SORT = 2,        /* voxelize + all radix sort passes + unique                  */
    GSC_STAGE_OCCUPANCY = 3,   /* the occupancy-byte kernel                                  */
    GSC_STAGE_PRELUDE = 4,     /* the first-level RAHT schedule launch (encoder, transforms) */
    GSC_STAGE_RAHT_FWD1 = 5,   /* the forward RAHT launch: merge, every level, quantize      */
    GSC_STAGE_RAHT_FWD_TOP = 6,/* (unused: the upper levels run in the forward launch)       */
    GSC_STAGE_RAHT_INV1 = 7,   /* first-level inverse RAHT (dequantize + transform + rows)   */
    GSC_STAGE_RAHT_INV_TOP = 8,/* inverse RAHT of the upper tiling levels                    */
    GSC_STAGE_OCTREE_DEC = 9,  /* octree expansion, Morton decode, centres, level-1 schedule */
    GSC_STAGE_COUNT = 10
} gsc_stage;

gsc_status gsc_profile_events(int32_t stage, void *const *events, int32_t n_pairs);

/* Human-readable name of a status code (static string). */
const char *gsc_status_string(gsc_status s);

#ifdef __cplusplus
}
#endif
#endif /* GSC_H */
