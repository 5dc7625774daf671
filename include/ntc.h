/*
 * ntc.h - C ABI of the MI355X (gfx950) neural BC1 texture decode library.
 *
 * Method: Belcour & Benyoub, "Hardware Accelerated Neural Block Texture
 * Compression with Cooperative Vectors". A material is a pyramid of latent
 * textures T_k stored as BC1 (Sec. 3.1, latent BC1 compression); a pixel at
 * coordinate uv is decoded by sampling every T_k bilinearly (Sec. 3.3),
 * concatenating the colours with uv into x and evaluating a small MLP
 * f(x) (Sec. 3.1, network architecture). The paper evaluates the MLP on
 * matrix engines over pixel tiles grouped by MLP (Sec. 4).
 *
 * Conventions for every entry point:
 *   - Pointers marked [device] are HIP device (or managed) memory, [host] are
 *     host memory read only during the call. The caller owns all memory; the
 *     library never allocates, frees or synchronises, and never prints.
 *   - `stream` is a hipStream_t (NULL = the null stream). Work is enqueued on
 *     it and the call returns without waiting; every launch is
 *     stream-ordered and contains no memset/memcpy nodes, so it can be
 *     captured into a HIP graph.
 *   - Arguments are validated on the host before anything is enqueued; on
 *     any error nothing is enqueued and a status other than NTC_OK is
 *     returned (ntc_last_error() then holds a message for this thread).
 *   - Outputs are fully overwritten. Inputs are never written.
 *
 * Feature layout (Sec. 3.1): x = [c_0.rgb, c_1.rgb, ..., c_{K-1}.rgb, u, v],
 * so dims[0] of every MLP must be 3 * n_levels + 2.
 * Texel centres sit at (i + 1/2) / W; level k is sampled at
 * x = u W_k - 1/2 + shift[k][0] texels (likewise y), which realises the
 * half-texel shift of the second and fourth textures (Sec. 3.1, variants)
 * when shift = {0, 1/2, 0, 1/2}.
 * Activations: ReLU on hidden layers, sigmoid on the output layer.
 */
#ifndef NTC_H_
#define NTC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NTC_MAX_LEVELS 4
#define NTC_MAX_LAYERS 5
#define NTC_MAX_CLASSIFY_MATERIALS 4096
#define NTC_MAX_MIPS 12
#define NTC_MAX_ANISO 16

typedef enum {
    NTC_OK = 0,
    NTC_E_NULL = 1,        /* a required pointer is NULL */
    NTC_E_SHAPE = 2,       /* inconsistent or out-of-range sizes */
    NTC_E_UNSUPPORTED = 3, /* valid request that the library does not implement */
    NTC_E_WORKSPACE = 4,   /* workspace / packed buffer too small */
    NTC_E_HIP = 5,         /* a HIP launch or runtime call failed */
    NTC_E_ALIGN = 6        /* a device pointer is not suitably aligned */
} ntc_status;

/* Arithmetic / storage types. */
typedef enum { NTC_F32 = 0, NTC_F16 = 1, NTC_BF16 = 2, NTC_FP8_E4M3 = 3 } ntc_dtype;

typedef enum { NTC_LATENT_BC1 = 0, NTC_LATENT_F32 = 1 } ntc_latent_fmt;

typedef enum { NTC_CLAMP = 0, NTC_WRAP = 1 } ntc_address;

/* Latent pyramid (Sec. 3.1). For NTC_LATENT_BC1, data[k] holds
 * (height[k]/4) x (width[k]/4) little-endian 64-bit BC1 blocks, block-row
 * major [device, 8-byte aligned]: bits 0-15 endpoint c0 (RGB565: red 11-15,
 * green 5-10, blue 0-4), bits 16-31 endpoint c1, bits 32-63 the 2-bit index
 * of texel (x, y) of the block at bit 32 + 2 (4y + x). c0 > c1 selects the
 * four-colour palette {e0, e1, (2e0+e1)/3, (e0+2e1)/3}, otherwise
 * {e0, e1, (e0+e1)/2, black} (Khronos BC1, cited in Sec. 3.1).
 * For NTC_LATENT_F32, data[k] is float [height][width][3] [device, 4-byte
 * aligned] of continuous latent values. Sizes: 4 <= width, height <= 16384,
 * multiples of 4 for BC1. */
typedef struct {
    int32_t n_levels;              /* 1 .. NTC_MAX_LEVELS */
    int32_t format;                /* ntc_latent_fmt */
    int32_t address;               /* ntc_address */
    int32_t reserved;              /* must be 0 */
    int32_t width[NTC_MAX_LEVELS];
    int32_t height[NTC_MAX_LEVELS];
    float shift[NTC_MAX_LEVELS][2];/* sampling offset in texels, |shift| <= 1 */
    const void *data[NTC_MAX_LEVELS];
} ntc_latents;

/* MLP (Sec. 3.1; widths as in Table 1): n_layers linear layers, layer l maps
 * dims[l] -> dims[l+1]. W[l] is float [dims[l+1]][dims[l]] row-major and
 * b[l] float [dims[l+1]] [device, FP32 master copy]. Limits: dims[0] =
 * 3 n_levels + 2 <= 14; 2 <= n_layers <= NTC_MAX_LAYERS; hidden widths all
 * equal and one of 16, 32, 64; 1 <= dims[n_layers] <= 16. */
typedef struct {
    int32_t n_layers;
    int32_t dims[NTC_MAX_LAYERS + 1];
    const float *W[NTC_MAX_LAYERS];
    const float *b[NTC_MAX_LAYERS];
} ntc_mlp;

/* Tile configuration of the MFMA decode. Zero fields pick defaults.
 *   waves_per_cu : workgroups (one wave each) launched per compute unit
 *                  (1..1024); each walks every grid-th span, so more than
 *                  the resident count trades weight reloads for balance
 *   tiles_per_iter: 64-pixel tiles a wave stages together (a span) before
 *                   running the MLP on them; fixed per network shape when
 *                   the library is compiled (by default 4 for 64-wide
 *                   networks of four or more layers and for the 64-wide
 *                   BF16 / E4M3 decodes, 8 otherwise); other values give
 *                   NTC_E_UNSUPPORTED
 *   stage_capacity: texels a wave may stage in LDS per span (64..4096,
 *                   default 1024); spans whose footprint is larger fall back
 *                   to direct block fetches. */
typedef struct {
    int32_t waves_per_cu;
    int32_t tiles_per_iter;
    int32_t stage_capacity;
    int32_t reserved;
} ntc_tile_cfg;

/* Human-readable name of a status code (static string). */
const char *ntc_status_string(ntc_status s);

/* Detail of the last error returned on this thread (static per-thread
 * buffer, empty if none). */
const char *ntc_last_error(void);

/* Library version as 10000 * major + 100 * minor + patch. */
int32_t ntc_version(void);

/* Bytes of the packed weight image of `mlp` for compute type `compute`
 * (NTC_F32, NTC_F16, NTC_BF16 or NTC_FP8_E4M3). [host] */
ntc_status ntc_mlp_pack_size(const ntc_mlp *mlp, int32_t compute, size_t *bytes);

/* Write the packed weight image used by ntc_decode: weights converted to
 * `compute`, padded to the matrix-core tile shapes and reordered so that
 * consecutive layers chain in registers; biases kept in FP32.
 * For NTC_F16, hidden neuron i of layer l is stored scaled by 2^-e(l, i),
 * e >= 0 chosen from an interval bound so that its pre-activation is at
 * most 1 whenever the latent values and u, v lie in [0, 1] (the weights
 * and biases absorb the powers of two, so the network is unchanged); the
 * decode then applies ReLU as the [0, 1] clamp of the FP16 conversion on
 * spans whose coordinates lie in the unit square, and the max-based ReLU
 * elsewhere. The output layer keeps e = 0, so its weights take the factor
 * 2^e of their input neuron; if a bound exceeds 2^10, or a scaled output
 * weight would exceed 2^15 (FP16 holds at most 65504), the image is left
 * unscaled and every span uses the max-based ReLU.
 * For NTC_FP8_E4M3, per-layer scales are powers of two computed on the
 * device: s_w = 2^floor(log2(448 / max|W_l|)); for the first layer's inputs
 * s_a = 2^floor(log2(448 / max(act_amax[0], 1))) (latent values reach 1),
 * the coordinates saturating at 448 / s_a; for hidden activations
 * s_a = 2^floor(log2(256 / act_amax[l])), their scaled values clamped to
 * [0, 256] (ReLU and clamp in one FP16 conversion, then a scaled FP16 ->
 * E4M3 conversion). Scaled values thus stay within E4M3's +-448, and the
 * factor that maps a layer's accumulator to the next layer's scaled input
 * / 256 is itself a power of two (the decode applies it as the matrix
 * instruction's E8M0 block scale). act_amax [device, n_layers
 * floats] must hold the largest |input| of every layer (see
 * ntc_calibrate_fp8). Otherwise act_amax is ignored. packed [device,
 * 256-byte aligned]. */
ntc_status ntc_mlp_pack(const ntc_mlp *mlp, int32_t compute, const float *act_amax,
                        void *packed, size_t bytes, void *stream);

/* FP8 range calibration: act_amax[l] = max over the n samples of |input of
 * layer l| (the feature vector for l = 0, the ReLU output of layer l-1
 * otherwise), evaluated with the plain FP32 decode [device, n_layers
 * floats, overwritten]. packed_f32 is the NTC_F32 image of `mlp` written by
 * ntc_mlp_pack; uv float [n][2] [device, 8-byte aligned], n >= 1. */
ntc_status ntc_calibrate_fp8(const ntc_latents *lat, const ntc_mlp *mlp, const void *packed_f32,
                             const float *uv, int64_t n, float *act_amax, void *stream);

/* Fused decode (Sec. 3.1 + Sec. 3.3 + Sec. 4): out[s] = f(x(uv[s])) for
 * s < n. compute selects the arithmetic: NTC_F32 (FP32: plain FMAs, one
 * pixel per lane, for BC1 latents; FP32 matrix cores, 32 samples per step,
 * for float latents and at most 4 layers), NTC_F16 (FP16 matrix cores, FP32
 * accumulation),
 * NTC_BF16 (BF16 matrix cores, FP32 accumulation) or NTC_FP8_E4M3 (E4M3
 * matrix cores with per-layer scales, FP32 accumulation). packed is the image written by ntc_mlp_pack for the same
 * compute type. uv float [n][2] [device, 8-byte aligned]; out [n][C]
 * with C = dims[n_layers] of out_dtype NTC_F32 or NTC_F16 [device, 16-byte
 * aligned]. n may be 0 (nothing is enqueued). BC1 latents only for
 * NTC_F16 / NTC_BF16 / NTC_FP8_E4M3. cfg may be NULL. */
ntc_status ntc_decode(const ntc_latents *lat, const ntc_mlp *mlp, int32_t compute, const void *packed,
                      const float *uv, int64_t n, void *out, int32_t out_dtype,
                      const ntc_tile_cfg *cfg, void *stream);

/* Workspace bytes needed by ntc_decode_backward for these shapes. [host] */
ntc_status ntc_decode_backward_workspace(const ntc_latents *lat, const ntc_mlp *mlp, int64_t n,
                                         size_t *bytes);

/* Backward of the FP32 decode (Sec. 3.2: gradients pass through the MLP into
 * the latent elements) for continuous latents (NTC_LATENT_F32): given
 * grad_out = dL/dout float [n][C] [device], writes
 *   grad_W[l] float [dims[l+1]][dims[l]], grad_b[l] float [dims[l+1]],
 *   grad_latents[k] float [height[k]][width[k]][3]          [all device]
 * (arrays of n_layers / n_levels device pointers [host]). Activations are
 * recomputed per tile of 32 samples with FP32 matrix-core products. Weight
 * gradients are summed per wavefront in FP32 and across wavefronts in FP64
 * (the same inputs give the same bits); latent gradients are accumulated
 * per spatial bin of samples in LDS and then with FP32 atomics (their
 * summation order is not deterministic). workspace [device, 256-byte
 * aligned] of at least ntc_decode_backward_workspace bytes (it grows with
 * n: 4 (3 n_levels + 1) bytes per sample plus the partial sums). */
ntc_status ntc_decode_backward(const ntc_latents *lat, const ntc_mlp *mlp, const float *uv, int64_t n,
                               const float *grad_out, float *const *grad_W, float *const *grad_b,
                               float *const *grad_latents, void *workspace, size_t ws_bytes,
                               void *stream);

/* ------------------------------------------------------------------------
 * Mip-mapped latents and filtered sampling (Sec. 3.2: every mip of a latent
 * texture is its own BC1 texture; Sec. 3.3: the latents are fetched with
 * trilinear or anisotropic filtering).
 * ---------------------------------------------------------------------- */
typedef enum { NTC_FILTER_TRILINEAR = 1, NTC_FILTER_ANISOTROPIC = 2 } ntc_filter;

typedef struct {
    int32_t n_levels;                           /* 1 .. NTC_MAX_LEVELS */
    int32_t n_mips[NTC_MAX_LEVELS];             /* 1 .. NTC_MAX_MIPS */
    int32_t width[NTC_MAX_LEVELS];              /* mip 0, texels */
    int32_t height[NTC_MAX_LEVELS];
    float shift[NTC_MAX_LEVELS][2];             /* sampling offset in texels of each mip, |shift| <= 1 */
    const void *data[NTC_MAX_LEVELS][NTC_MAX_MIPS]; /* BC1 blocks of mip m: (width >> m) x (height >> m)
                                                   texels, multiples of 4 [device, 8-byte aligned] */
} ntc_latent_mips;

/* Filtered decode with FP16 matrix cores: out[s] = f(x(uv[s])) where the
 * features of level k are filtered over its mip chain, clamp-to-edge
 * addressing inside each mip. duv float [n][4] [device, 16-byte aligned]
 * holds the screen derivatives (du/dx, dv/dx, du/dy, dv/dy) of each
 * sample. With the footprint axes measured in texels of mip 0,
 * Px = |(du/dx W, dv/dx H)|, Py = |(du/dy W, dv/dy H)|:
 *   NTC_FILTER_TRILINEAR: lod = log2 max(Px, Py), clamped to [0, n_mips - 1];
 *     the bilinear samples of mips floor(lod) and floor(lod) + 1 are blended
 *     by the fraction of lod;
 *   NTC_FILTER_ANISOTROPIC: N = min(ceil(Pmax / Pmin), max_aniso) trilinear
 *     samples at lod = log2(Pmax / N) along the longer axis, at
 *     uv + (i / (N + 1) - 1/2) (du, dv) for i = 1..N, averaged. N is
 *     decided in FP32 as the smallest n with n^2 Pmin^2 >= Pmax^2, the
 *     squared lengths and that product rounded as FP32 operations (no fused
 *     multiply-add); this is min(ceil(Pmax / Pmin), max_aniso) except where
 *     Pmax / Pmin lies within FP32 rounding of an integer.
 * max_aniso in 1..NTC_MAX_ANISO. packed is the NTC_F16 image of mlp; uv,
 * out and out_dtype as for ntc_decode. */
ntc_status ntc_decode_filtered(const ntc_latent_mips *lat, const ntc_mlp *mlp, const void *packed, const float *uv,
                               const float *duv, int64_t n, void *out, int32_t out_dtype, int32_t filter,
                               int32_t max_aniso, void *stream);

/* ------------------------------------------------------------------------
 * Trainable BC1 latents (Sec. 3.2, Eqs. 1-3: endpoints and interpolation
 * weights kept as floats, a sigmoid, then quantisation to the BC1 field
 * widths that gradients pass through unchanged).
 *
 * One level of width x height texels (multiples of 4, at most 16384) is a
 * parameter array params float [height/4][width/4][22] [device]: per block
 * the logits of endpoint 0 (r, g, b), endpoint 1 (r, g, b) and of the 16
 * texel weights (texel (x, y) of the block at index 4 y + x). Codes:
 * E = round(sigmoid(e) (2^b - 1)) with b = 5, 6, 5 bits for r, g, b and
 * w = round(sigmoid(alpha) 3); a texel's value per channel is
 * ((3 - w) E0 + w E1) / (3 (2^b - 1)), the four-colour BC1 palette. A code
 * is the number of rounding midpoints (k + 1/2) / (2^b - 1) whose logit
 * (correctly rounded to FP32) is at or below the parameter: the rounding of
 * the sigmoid, with a logit equal to such an FP32 constant rounding up.
 * NaN parameters give code 0. All three calls are stream-ordered and
 * allocate nothing.
 * ---------------------------------------------------------------------- */

/* texels float [height][width][3] [device] = the quantised texel values
 * (each the FP32 value nearest the exact rational, as ntc_bc1_decode_texels
 * gives for the exported blocks). */
ntc_status ntc_qat_texels(const float *params, int32_t width, int32_t height, float *texels, void *stream);

/* grad_params float [height/4][width/4][22] [device, overwritten] from
 * grad_texels = dL/dtexels float [height][width][3] [device], with the
 * quantisation passed through: dL/dE0 = sum over the block's texels of
 * (1 - w/3) g, dL/dE1 = sum of (w/3) g, dL/d(w/3) = sum over channels of
 * (E1 - E0) g (E as values in [0, 1]), each times sigmoid'(logit). */
ntc_status ntc_qat_backward(const float *params, int32_t width, int32_t height, const float *grad_texels,
                            float *grad_params, void *stream);

/* blocks uint64 [height/4][width/4] [device, 8-byte aligned] = BC1 blocks
 * whose decode equals ntc_qat_texels: four-colour mode, the larger 565
 * endpoint first (weights mirrored when the endpoints swap), and when both
 * endpoints are equal every index 0. */
ntc_status ntc_qat_export_bc1(const float *params, int32_t width, int32_t height, uint64_t *blocks, void *stream);

/* ------------------------------------------------------------------------
 * Classification of a frame by material (Sec. 4 "Tile-based
 * classification", Algorithm 1): the screen is cut into 8x4-pixel tiles; a
 * tile whose valid pixels all use one material and number more than 16 is
 * "simple" and is decoded as it stands, the pixels of every other tile are
 * regrouped by material. The result feeds the batched decode.
 * ---------------------------------------------------------------------- */

/* Workspace bytes for ntc_classify. [host] */
ntc_status ntc_classify_workspace(int32_t width, int32_t height, int32_t n_mats, size_t *bytes);

/* mat_ids uint16 [height][width] [device]: the material (MLP) of each pixel;
 * ids >= n_mats mark pixels without a neural material. width, height in
 * 1..32768 (fewer than 2^31 pixels); n_mats in 1..NTC_MAX_CLASSIFY_MATERIALS.
 * Tiles are numbered row-major, tile (tx, ty) covering pixels
 * [8 tx, 8 tx + 8) x [4 ty, 4 ty + 4) (clipped at the frame edge).
 * Outputs [device, overwritten]:
 *   pixel_list  int32 [width height]: the indices y width + x of the valid
 *               pixels, grouped by material in material order; inside a
 *               material first the pixels of its simple tiles, then its
 *               other pixels, each part in tile order and row-major inside
 *               a tile (entries past the valid count are left untouched);
 *   mat_offsets int32 [n_mats + 1]: material m occupies
 *               [mat_offsets[m], mat_offsets[m + 1]); mat_offsets[n_mats] is
 *               the number of valid pixels;
 *   mat_simple  int32 [n_mats]: how many of them come from simple tiles;
 *   tile_class  uint8 [tiles] or NULL: 0 no valid pixel, 1 simple, 2 other.
 * The order is fixed (no atomics decide it): the same input gives the same
 * lists. workspace [device, 256-byte aligned] of ntc_classify_workspace
 * bytes. */
ntc_status ntc_classify(const uint16_t *mat_ids, int32_t width, int32_t height, int32_t n_mats, int32_t *pixel_list,
                        int32_t *mat_offsets, int32_t *mat_simple, uint8_t *tile_class, void *workspace,
                        size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, per-frame serving loops, harnesses that forbid allocation): the
 * same classification as ntc_classify, with the same arguments and outputs
 * but no workspace argument. The counts that ntc_classify keeps in its
 * workspace live in a file-scope device array of 8 MiB, one per GPU the
 * library runs on, held until the process ends; its device address is
 * looked up on the first call on each device. The call allocates and frees
 * nothing. Frames needing more than 8 MiB of counts,
 * 8 n_mats (ceil(tiles / 128) + 1) bytes with tiles = ceil(width / 8)
 * ceil(height / 4) (for example 4096 x 4096 with more than 255 materials),
 * are rejected with NTC_E_WORKSPACE. Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (different streams,
 * or threads) race and give wrong lists; calls ordered on one stream do
 * not. */
ntc_status ntc_classify_noalloc(const uint16_t *mat_ids, int32_t width, int32_t height, int32_t n_mats,
                                int32_t *pixel_list, int32_t *mat_offsets, int32_t *mat_simple,
                                uint8_t *tile_class, void *stream);

/* uv[i] = uv_image[pixel_list[i]] for i < n: uv_image float [pixels][2],
 * uv float [n][2] [device, 8-byte aligned]. */
ntc_status ntc_gather_uv(const float *uv_image, const int32_t *pixel_list, int64_t n, float *uv, void *stream);

/* image[pixel_list[i]][c] = rows[i][c] for i < n, c < channels (1..16), dtype
 * NTC_F32 or NTC_F16 [device]. */
ntc_status ntc_scatter_rows(const void *rows, const int32_t *pixel_list, int64_t n, int32_t channels, int32_t dtype,
                            void *image, void *stream);

/* ------------------------------------------------------------------------
 * Many materials in one launch (Sec. 4: pixels are grouped by MLP so that
 * a workgroup runs one set of weights; Alg. 1 builds per-MLP tile groups).
 * ---------------------------------------------------------------------- */
typedef struct {
    ntc_latents lat;   /* BC1 latents [device] */
    ntc_mlp mlp;       /* shapes (dims, n_layers); W / b may be NULL */
    const void *packed;/* NTC_F16 packed image of this material [device] */
    const float *uv;   /* [n][2] [device] (with pixel_index: the uv image, [image_pixels][2]) */
    int64_t n;
    void *out;         /* [n][C] [device] (with pixel_index: the output image, [image_pixels][C]) */
    int32_t out_dtype; /* NTC_F32 or NTC_F16 */
    int32_t reserved;
    /* Optional [device] int32 [n]: sample s is pixel pixel_index[s] of images
     * of image_pixels pixels: its uv is read from uv[pixel_index[s]] and its
     * output written to out[pixel_index[s]] (the per-material lists of
     * ntc_classify feed the decode directly). An index outside
     * 0..image_pixels-1 reads uv (0, 0) and writes nothing. NULL: uv and out
     * are the material's own [n] arrays. image_pixels * C * (4 or 2) must be
     * below 2^31. */
    const int32_t *pixel_index;
    int64_t image_pixels;
} ntc_material;

/* Batch options. item_pixels: pixels per work item (multiple of 64,
 * 64..65536, 0 = 4096); waves_per_cu as in ntc_tile_cfg. */
typedef struct {
    int32_t item_pixels;
    int32_t waves_per_cu;
    int32_t stage_capacity;
    int32_t n_cus;      /* compute units to size the grid for (0 = 256) */
} ntc_batch_cfg;

/* Bytes of the plan image for this batch. [host] */
ntc_status ntc_batched_plan_size(const ntc_material *mats, int32_t n_mats, const ntc_batch_cfg *cfg,
                                 size_t *bytes);

/* Build the plan image [host buffer of plan_size bytes]: the material
 * table and a work list of (material, pixel range) items, grouped by MLP
 * shape and assigned to persistent waves by longest-processing-time-first
 * bin packing. The caller copies it to device memory (any 256-byte aligned
 * buffer) before ntc_decode_batched; device pointers inside are those of
 * `mats`. */
ntc_status ntc_batched_plan(const ntc_material *mats, int32_t n_mats, const ntc_batch_cfg *cfg,
                            void *plan_host, size_t bytes);

/* Decode every material of the plan in one persistent launch. plan_host is
 * the host image (read for the launch size only), plan_dev its device copy. */
ntc_status ntc_decode_batched(const void *plan_host, const void *plan_dev, size_t bytes, void *stream);

/* ------------------------------------------------------------------------
 * Test export: BC1 texel decode of one level (Sec. 3.1 blend).
 * numer [device, may be NULL] uint16 [H][W][3]: exact numerators of the
 * channel values over 6 (2^b - 1), i.e. over 186 for red and blue and 378
 * for green. out [device, may be NULL] float [H][W][3]: the value
 * numer / denominator rounded once to FP32.
 * ---------------------------------------------------------------------- */
ntc_status ntc_bc1_decode_texels(const ntc_latents *lat, int32_t level, float *out, uint16_t *numer,
                                 void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NTC_H_ */
