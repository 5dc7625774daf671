/*
 * FP64 CPU oracle of the neural BC1 texture decode.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow definition that the
 * GPU library is checked against. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it. It shares no code, header,
 * table or constant with the GPU library and includes nothing from it.
 *
 * What it computes (Belcour & Benyoub, "Hardware Accelerated Neural Block
 * Texture Compression with Cooperative Vectors"):
 *   - Sec. 3.1, latent BC1 compression: every texel of a latent texture is a
 *     blend (1-a) e0 + a e1 of two RGB565 endpoints shared by a 4x4 block,
 *     with a 2-bit blend index per texel; the block layout and the
 *     three-colour mode follow the Khronos BC1 definition the paper cites.
 *   - Sec. 3.1 (architecture) and Sec. 3.3: each latent k is sampled at uv
 *     with bilinear filtering, the colours are concatenated into x and an
 *     MLP maps x to the output channels f = f(x).
 *   - Sec. 3.1, variants: the second and fourth textures are shifted by half
 *     a texel.
 *   - Sec. 3.2: gradients flow through the MLP into every latent element.
 *
 * Readings of what the paper leaves open (activations, texel centres,
 * address mode, feature order, precision emulation) are those of the
 * project's design notes; each is restated next to the code that uses it.
 *
 * All arithmetic is IEEE double. Inputs given as float32 by callers are
 * widened exactly before they get here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_LEVELS 8
#define OR_MAX_LAYERS 8
#define OR_MAX_DIM 128

/* One latent texture. format 0: BC1 blocks, uint64 [(H/4)][(W/4)], block
 * row-major, little-endian words. format 1: double grid [H][W][3]. */
typedef struct {
    int32_t width, height, format, pad_;
    const void *data;
    double shift_x, shift_y; /* texel units */
} oracle_level;

typedef struct {
    int32_t n_layers;
    int32_t dims[OR_MAX_LAYERS + 1];
    const double *W[OR_MAX_LAYERS]; /* [dims[l+1]][dims[l]] row-major */
    const double *b[OR_MAX_LAYERS];
    int32_t precision;              /* 0 exact, 1 round to binary16, 2 round to E4M3 with scales,
                                       3 as 2 with hidden activations through binary16 */
    const double *w_scale;          /* [n_layers], precision 2 and 3 only */
    const double *a_scale;          /* [n_layers], precision 2 and 3 only */
} oracle_mlp;

/* ------------------------------------------------------------------------
 * Rounding to the narrow formats, written from the format definitions:
 * round-to-nearest, ties to even, at the spacing of the binade of |x|.
 * ---------------------------------------------------------------------- */

/* IEEE 754 binary16: 10 fraction bits, exponent range [-14, 15], subnormal
 * spacing 2^-24, largest finite 65504; values that round beyond it become
 * infinite. */
double oracle_round_f16(double x) {
    if (x != x || x == 0.0) return x;
    double a = fabs(x);
    int e;
    frexp(a, &e);          /* a = m * 2^e, m in [0.5, 1) => floor(log2 a) = e - 1 */
    int ex = e - 1;
    if (ex < -14) ex = -14;
    double q = ldexp(1.0, ex - 10);
    double r = nearbyint(a / q) * q; /* default rounding mode: ties to even */
    if (r > 65504.0) r = INFINITY;
    return x < 0 ? -r : r;
}

/* OCP 8-bit E4M3 ("FN": no infinities): 3 fraction bits, exponent bias 7,
 * smallest normal 2^-6, subnormal spacing 2^-9, largest finite 448. The
 * conversion used by the quantised path saturates: results beyond 448 in
 * magnitude are 448. */
double oracle_round_e4m3_sat(double x) {
    if (x != x || x == 0.0) return x;
    double a = fabs(x);
    int e;
    frexp(a, &e);
    int ex = e - 1;
    if (ex < -6) ex = -6;
    double q = ldexp(1.0, ex - 3);
    double r = nearbyint(a / q) * q;
    if (r > 448.0) r = 448.0;
    return x < 0 ? -r : r;
}

/* ------------------------------------------------------------------------
 * BC1 texel (Sec. 3.1 latent BC1 compression; Khronos BC1 layout).
 * Block word: bits 0-15 endpoint c0, bits 16-31 endpoint c1, bits 32-63
 * sixteen 2-bit indices, texel (x, y) of the block at index 4y + x.
 * Endpoint RGB565: red bits 11-15, green 5-10, blue 0-4; a b-bit field E
 * stands for the value E / (2^b - 1).
 * c0 > c1 (four colours): indices 0,1,2,3 blend with a = 0, 1, 1/3, 2/3.
 * c0 <= c1 (three colours): indices 0,1,2 blend with a = 0, 1, 1/2 and
 * index 3 is black.
 * The value of channel ch is num[ch] / den[ch] exactly.
 * ---------------------------------------------------------------------- */
void oracle_bc1_texel(const uint64_t *blocks, int32_t width, int32_t i, int32_t j,
                      int32_t num[3], int32_t den[3]) {
    uint64_t blk = blocks[(int64_t)(j / 4) * (width / 4) + (i / 4)];
    uint32_t c0 = (uint32_t)(blk & 0xFFFFu);
    uint32_t c1 = (uint32_t)((blk >> 16) & 0xFFFFu);
    uint32_t indices = (uint32_t)(blk >> 32);
    int pos = 4 * (j % 4) + (i % 4);
    uint32_t idx = (indices >> (2 * pos)) & 3u;
    int e0[3] = {(int)(c0 >> 11) & 31, (int)(c0 >> 5) & 63, (int)c0 & 31};
    int e1[3] = {(int)(c1 >> 11) & 31, (int)(c1 >> 5) & 63, (int)c1 & 31};
    int maxv[3] = {31, 63, 31};
    for (int ch = 0; ch < 3; ++ch) {
        if (c0 > c1) {
            /* a = t / 3 with t = 0, 3, 1, 2 for indices 0..3 */
            static const int t_of_idx[4] = {0, 3, 1, 2};
            int t = t_of_idx[idx];
            num[ch] = (3 - t) * e0[ch] + t * e1[ch];
            den[ch] = 3 * maxv[ch];
        } else if (idx == 3) {
            num[ch] = 0;
            den[ch] = 1;
        } else {
            /* a = t / 2 with t = 0, 2, 1 for indices 0..2 */
            static const int t_of_idx3[3] = {0, 2, 1};
            int t = t_of_idx3[idx];
            num[ch] = (2 - t) * e0[ch] + t * e1[ch];
            den[ch] = 2 * maxv[ch];
        }
    }
}

/* Every texel of one BC1 level: num/den int32 [H][W][3], val = num/den. */
void oracle_bc1_level(const uint64_t *blocks, int32_t width, int32_t height,
                      int32_t *num, int32_t *den, double *val) {
    for (int32_t j = 0; j < height; ++j)
        for (int32_t i = 0; i < width; ++i) {
            int32_t n[3], d[3];
            oracle_bc1_texel(blocks, width, i, j, n, d);
            for (int ch = 0; ch < 3; ++ch) {
                int64_t o = ((int64_t)j * width + i) * 3 + ch;
                if (num) num[o] = n[ch];
                if (den) den[o] = d[ch];
                if (val) val[o] = (double)n[ch] / (double)d[ch];
            }
        }
}

static double texel_value(const oracle_level *lv, int32_t i, int32_t j, int ch) {
    if (lv->format == 0) {
        int32_t n[3], d[3];
        oracle_bc1_texel((const uint64_t *)lv->data, lv->width, i, j, n, d);
        return (double)n[ch] / (double)d[ch];
    }
    return ((const double *)lv->data)[((int64_t)j * lv->width + i) * 3 + ch];
}

/* Address mode 0: clamp to edge; 1: wrap (repeat). */
static int32_t address(int32_t i, int32_t n, int32_t mode) {
    if (mode == 1) {
        int32_t r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Bilinear footprint of one sample on one level (Sec. 3.3: the latents are
 * bilinearly filtered). Texel centres sit at (i + 1/2) / W; the level's
 * shift (Sec. 3.1 variants, half a texel on textures 2 and 4) moves the
 * sampling position by s texels: x = u W - 1/2 + s. Taps (i0, j0) ..
 * (i0+1, j0+1) with weights (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy. */
typedef struct {
    int32_t ti[4], tj[4];
    double w[4];
} footprint;

static void bilinear_footprint(const oracle_level *lv, double u, double v, int32_t mode,
                               footprint *fp) {
    double x = u * lv->width - 0.5 + lv->shift_x;
    double y = v * lv->height - 0.5 + lv->shift_y;
    double fx0 = floor(x), fy0 = floor(y);
    double fx = x - fx0, fy = y - fy0;
    int32_t i0 = (int32_t)fx0, j0 = (int32_t)fy0;
    for (int t = 0; t < 4; ++t) {
        int di = t & 1, dj = t >> 1;
        fp->ti[t] = address(i0 + di, lv->width, mode);
        fp->tj[t] = address(j0 + dj, lv->height, mode);
        fp->w[t] = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy);
    }
}

/* Feature vector x = [c_0 .. c_{K-1}, u, v] (Sec. 3.1: concatenation of the
 * sampled latent colours; u and v are appended). */
static void features_one(const oracle_level *lv, int32_t n_levels, int32_t mode,
                         double u, double v, double *x) {
    for (int k = 0; k < n_levels; ++k) {
        footprint fp;
        bilinear_footprint(&lv[k], u, v, mode, &fp);
        for (int ch = 0; ch < 3; ++ch) {
            double c = 0.0;
            for (int t = 0; t < 4; ++t) c += fp.w[t] * texel_value(&lv[k], fp.ti[t], fp.tj[t], ch);
            x[3 * k + ch] = c;
        }
    }
    x[3 * n_levels] = u;
    x[3 * n_levels + 1] = v;
}

void oracle_features(const oracle_level *lv, int32_t n_levels, int32_t mode,
                     const double *uv, int64_t n, double *x, int32_t threads) {
    int32_t nf = 3 * n_levels + 2;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (int64_t s = 0; s < n; ++s) features_one(lv, n_levels, mode, uv[2 * s], uv[2 * s + 1], x + s * nf);
}

/* Quantised input of layer l. Precision 3 takes the activations of the
 * hidden layers (l > 0, non-negative after ReLU) to E4M3 in two steps: the
 * scaled value divided by 256 is clamped to [0, 1] and rounded to binary16,
 * and that value times 256 (at most 256, so no saturation) is rounded to
 * E4M3; the first layer's inputs are rounded as in precision 2. */
static double quant_act(const oracle_mlp *m, int l, double a) {
    if (m->precision == 1) return oracle_round_f16(a);
    if (m->precision == 3 && l > 0) {
        double t = a * m->a_scale[l] / 256.0;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        return oracle_round_e4m3_sat(256.0 * oracle_round_f16(t));
    }
    if (m->precision >= 2) return oracle_round_e4m3_sat(a * m->a_scale[l]);
    return a;
}

static double quant_w(const oracle_mlp *m, int l, double w) {
    if (m->precision == 1) return oracle_round_f16(w);
    if (m->precision >= 2) return oracle_round_e4m3_sat(w * m->w_scale[l]);
    return w;
}

/* MLP f(x) (Sec. 3.1): hidden layers h = max(0, W h + b), output layer
 * f = 1 / (1 + exp(-(W h + b))). With precision 1 the layer inputs and the
 * weights are first rounded to binary16; with precision 2 and 3 they are
 * scaled and rounded to E4M3 (quant_act, quant_w) and the dot product is
 * divided by both scales. The bias and the accumulation stay exact in every
 * case. If z is not NULL the
 * pre-activations of every layer are stored there, layer after layer. */
static void mlp_one(const oracle_mlp *m, const double *x, double *f, double *z_all,
                    double *amax) {
    double h[OR_MAX_DIM], hn[OR_MAX_DIM];
    int32_t d0 = m->dims[0];
    for (int k = 0; k < d0; ++k) h[k] = x[k];
    int64_t zoff = 0;
    for (int l = 0; l < m->n_layers; ++l) {
        int32_t di = m->dims[l], dout = m->dims[l + 1];
        if (amax)
            for (int k = 0; k < di; ++k)
                if (fabs(h[k]) > amax[l]) amax[l] = fabs(h[k]);
        double hq[OR_MAX_DIM];
        for (int k = 0; k < di; ++k) hq[k] = quant_act(m, l, h[k]);
        for (int o = 0; o < dout; ++o) {
            double acc = 0.0;
            const double *wr = m->W[l] + (int64_t)o * di;
            for (int k = 0; k < di; ++k) acc += quant_w(m, l, wr[k]) * hq[k];
            if (m->precision >= 2) acc /= (m->w_scale[l] * m->a_scale[l]);
            acc += m->b[l][o];
            if (z_all) z_all[zoff + o] = acc;
            hn[o] = (l + 1 < m->n_layers) ? (acc > 0.0 ? acc : 0.0) : 1.0 / (1.0 + exp(-acc));
        }
        zoff += dout;
        for (int o = 0; o < dout; ++o) h[o] = hn[o];
    }
    for (int o = 0; o < m->dims[m->n_layers]; ++o) f[o] = h[o];
}

/* The MLP alone on given feature vectors: out[s] = f(x[s]), x [n][dims[0]]. */
void oracle_mlp_forward(const oracle_mlp *m, const double *x, int64_t n, double *out, int32_t threads) {
    int32_t d0 = m->dims[0], C = m->dims[m->n_layers];
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads > 0 ? threads : 1)
    for (int64_t s = 0; s < n; ++s) mlp_one(m, x + s * d0, out + s * C, NULL, NULL);
}

/* Full decode p(uv) = f(x(uv)) for n samples: out [n][C]. */
void oracle_decode(const oracle_level *lv, int32_t n_levels, int32_t mode, const oracle_mlp *m,
                   const double *uv, int64_t n, double *out, int32_t threads) {
    int32_t C = m->dims[m->n_layers];
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads > 0 ? threads : 1)
    for (int64_t s = 0; s < n; ++s) {
        double x[3 * OR_MAX_LEVELS + 2];
        features_one(lv, n_levels, mode, uv[2 * s], uv[2 * s + 1], x);
        mlp_one(m, x, out + s * C, NULL, NULL);
    }
}

/* Decode a subset of samples: out[r] = p(uv[index[r]]). */
void oracle_decode_index(const oracle_level *lv, int32_t n_levels, int32_t mode,
                         const oracle_mlp *m, const double *uv, const int64_t *index, int64_t n,
                         double *out, int32_t threads) {
    int32_t C = m->dims[m->n_layers];
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads > 0 ? threads : 1)
    for (int64_t r = 0; r < n; ++r) {
        double x[3 * OR_MAX_LEVELS + 2];
        int64_t s = index[r];
        features_one(lv, n_levels, mode, uv[2 * s], uv[2 * s + 1], x);
        mlp_one(m, x, out + r * C, NULL, NULL);
    }
}

/* Largest |input| of every layer over n samples (FP8 range calibration). */
void oracle_layer_amax(const oracle_level *lv, int32_t n_levels, int32_t mode, const oracle_mlp *m,
                       const double *uv, int64_t n, double *amax) {
    double f[OR_MAX_DIM];
    for (int l = 0; l < m->n_layers; ++l) amax[l] = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        double x[3 * OR_MAX_LEVELS + 2];
        features_one(lv, n_levels, mode, uv[2 * s], uv[2 * s + 1], x);
        mlp_one(m, x, f, NULL, amax);
    }
}

/* Gradient of sum_s sum_c g[s][c] f_c(uv_s) (Sec. 3.2: gradients pass through
 * the MLP into the latent elements), for float latent grids (format 1):
 *   d_L  = g * f (1 - f)                       (sigmoid output)
 *   d_l  = (W_{l+1}^T d_{l+1}) * [z_l > 0]     (ReLU, derivative 0 at 0)
 *   dW_l = sum_s d_l h_{l-1}^T,  db_l = sum_s d_l
 *   dx   = W_0^T d_0, and each latent texel receives the bilinear weight of
 *          its tap times dx of its channel (taps that clamp onto the same
 *          texel add up).
 * gW[l], gb[l] and glat[k] ([H][W][3]) are overwritten. Exact arithmetic
 * only (precision 0). threads > 1 sums per-thread partials in thread order. */
void oracle_backward(const oracle_level *lv, int32_t n_levels, int32_t mode, const oracle_mlp *m,
                     const double *uv, int64_t n, const double *g, double **gW, double **gb,
                     double **glat, int32_t threads) {
    if (threads < 1) threads = 1;
    int L = m->n_layers;
    int64_t wsz[OR_MAX_LAYERS], lsz[OR_MAX_LEVELS];
    int64_t wtot = 0, ltot = 0;
    for (int l = 0; l < L; ++l) {
        wsz[l] = (int64_t)m->dims[l] * m->dims[l + 1] + m->dims[l + 1];
        wtot += wsz[l];
    }
    for (int k = 0; k < n_levels; ++k) {
        lsz[k] = (int64_t)lv[k].width * lv[k].height * 3;
        ltot += lsz[k];
    }
    double *part = (double *)calloc((size_t)threads * (size_t)(wtot + ltot), sizeof(double));
    if (!part) return;
    int32_t C = m->dims[L];
#pragma omp parallel num_threads(threads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = part + (int64_t)tid * (wtot + ltot);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < n; ++s) {
            double u = uv[2 * s], v = uv[2 * s + 1];
            double x[3 * OR_MAX_LEVELS + 2];
            features_one(lv, n_levels, mode, u, v, x);
            double z[OR_MAX_LAYERS * OR_MAX_DIM], f[OR_MAX_DIM];
            mlp_one(m, x, f, z, NULL);
            /* layer inputs h_l and pre-activations z_l */
            const double *zl[OR_MAX_LAYERS];
            int64_t zo = 0;
            for (int l = 0; l < L; ++l) { zl[l] = z + zo; zo += m->dims[l + 1]; }
            double hin[OR_MAX_LAYERS][OR_MAX_DIM];
            for (int k = 0; k < m->dims[0]; ++k) hin[0][k] = x[k];
            for (int l = 1; l < L; ++l)
                for (int k = 0; k < m->dims[l]; ++k) hin[l][k] = zl[l - 1][k] > 0.0 ? zl[l - 1][k] : 0.0;
            double d[OR_MAX_DIM], dprev[OR_MAX_DIM];
            for (int c = 0; c < C; ++c) d[c] = g[s * C + c] * f[c] * (1.0 - f[c]);
            int64_t woff = wtot;
            for (int l = L - 1; l >= 0; --l) {
                int32_t di = m->dims[l], dout = m->dims[l + 1];
                woff -= wsz[l];
                double *gw = mine + woff, *gbias = gw + (int64_t)di * dout;
                for (int o = 0; o < dout; ++o) {
                    for (int k = 0; k < di; ++k) gw[(int64_t)o * di + k] += d[o] * hin[l][k];
                    gbias[o] += d[o];
                }
                for (int k = 0; k < di; ++k) {
                    double acc = 0.0;
                    for (int o = 0; o < dout; ++o) acc += m->W[l][(int64_t)o * di + k] * d[o];
                    dprev[k] = acc;
                }
                if (l > 0)
                    for (int k = 0; k < di; ++k) d[k] = zl[l - 1][k] > 0.0 ? dprev[k] : 0.0;
            }
            /* dprev now holds dx = W_0^T d_0 */
            int64_t loff = wtot;
            for (int k = 0; k < n_levels; ++k) {
                footprint fp;
                bilinear_footprint(&lv[k], u, v, mode, &fp);
                double *gl = mine + loff;
                for (int t = 0; t < 4; ++t)
                    for (int ch = 0; ch < 3; ++ch)
                        gl[((int64_t)fp.tj[t] * lv[k].width + fp.ti[t]) * 3 + ch] += fp.w[t] * dprev[3 * k + ch];
                loff += lsz[k];
            }
        }
    }
    /* reduce partials in thread order */
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        int64_t nw = (int64_t)m->dims[l] * m->dims[l + 1];
        for (int64_t e = 0; e < wsz[l]; ++e) {
            double acc = 0.0;
            for (int t = 0; t < threads; ++t) acc += part[(int64_t)t * (wtot + ltot) + off + e];
            if (e < nw) gW[l][e] = acc; else gb[l][e - nw] = acc;
        }
        off += wsz[l];
    }
    for (int k = 0; k < n_levels; ++k) {
        for (int64_t e = 0; e < lsz[k]; ++e) {
            double acc = 0.0;
            for (int t = 0; t < threads; ++t) acc += part[(int64_t)t * (wtot + ltot) + off + e];
            glat[k][e] = acc;
        }
        off += lsz[k];
    }
    free(part);
}

/* Smallest |pre-activation| over the hidden units of every sample: the
 * distance of the sample from a ReLU kink, where FP32 and FP64 evaluations
 * may take different derivative branches. */
void oracle_relu_margin(const oracle_level *lv, int32_t n_levels, int32_t mode, const oracle_mlp *m,
                        const double *uv, int64_t n, double *margin, int32_t threads) {
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads > 0 ? threads : 1)
    for (int64_t s = 0; s < n; ++s) {
        double x[3 * OR_MAX_LEVELS + 2], z[OR_MAX_LAYERS * OR_MAX_DIM], f[OR_MAX_DIM];
        features_one(lv, n_levels, mode, uv[2 * s], uv[2 * s + 1], x);
        mlp_one(m, x, f, z, NULL);
        double mg = INFINITY;
        int64_t off = 0;
        for (int l = 0; l + 1 < m->n_layers; ++l) {
            for (int k = 0; k < m->dims[l + 1]; ++k)
                if (fabs(z[off + k]) < mg) mg = fabs(z[off + k]);
            off += m->dims[l + 1];
        }
        margin[s] = mg;
    }
}

int32_t oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
