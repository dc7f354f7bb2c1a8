/*
 * niv_oracle.c -- plain FP64 CPU reference for the Neural Irradiance Volume.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct model
 * that the GPU library is checked against.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product path
 * never does.  It shares no source with the GPU library.
 *
 * What it follows (Coomans, Nazzaro et al., "Real-time Rendering with a
 * Neural Irradiance Volume", Eurographics 2026):
 *   - irradiance E(x,n), Eq. 1; diffuse shading rho/pi * E, Eq. 2 (Sec. 3);
 *   - the model: multi-level hash-grid encoding of x plus a ReLU MLP with a
 *     linear output (Sec. 4.1); per-frame scene variables frequency-encoded
 *     as extra inputs (Sec. 6);
 *   - training: relative L2 loss with a stop-gradient denominator, Eq. 3;
 *     Adam with an exponentially decaying learning rate (Sec. 4.5);
 *   - targets: Monte Carlo estimates of the indirect part of Eq. 1 with
 *     back-face culling and null-irradiance rejection (Sec. 4.5, App. H);
 *   - rendering: joint bilateral upsampling of a half-resolution query and
 *     dynamic ambient occlusion from the dynamic geometry only (Sec. 4.4).
 * Readings of points the paper leaves open are listed next to the code that
 * takes them.
 *
 * All arithmetic is double precision.  Compile with -ffp-contract=off so
 * that no multiply-add is fused except where fma() is written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Model configuration                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int n_levels;          /* L */
    int log2_T;            /* hash table size T = 2^log2_T */
    int n_features;        /* F, latent size per entry */
    double base_res;       /* N_min, coarsest resolution */
    double per_level_scale;/* b, growth factor between levels */
    int sh_bands;          /* direction encoding: sh_bands^2 real SH, 0 = none */
    int n_extra;           /* scene variables appended to the input */
    int extra_bands;       /* frequency bands per scene variable */
    int width;             /* hidden width */
    int n_hidden;          /* number of hidden layers */
    int n_out;             /* outputs (3 = RGB) */
    double aabb_min[3], aabb_max[3];
    int pos_bands;         /* positional code of x: 0 = none, else bands */
} orc_config;

/* Level table (Sec. 4.1, learned encodings).  Reading: the resolution of
 * level l is floor(N_min * b^l), taken with a tiny relative guard so that a
 * product that is mathematically an integer is not floored to the integer
 * below; a level is stored densely with (N+1)^3 entries when that fits in T,
 * otherwise it is a hash table of T entries.  Offsets are prefix sums.
 * Returns the total number of entries. */
int64_t orc_level_table(const orc_config *c, int64_t *res, int *dense,
                        int64_t *size, int64_t *offset)
{
    int64_t T = (int64_t)1 << c->log2_T, total = 0;
    for (int l = 0; l < c->n_levels; ++l) {
        double x = c->base_res * pow(c->per_level_scale, (double)l);
        int64_t N = (int64_t)floor(x * (1.0 + 0x1p-40));
        int64_t side = N + 1;
        int d = (side * side * side) <= T;
        int64_t sz = d ? side * side * side : T;
        if (res) res[l] = N;
        if (dense) dense[l] = d;
        if (size) size[l] = sz;
        if (offset) offset[l] = total;
        total += sz;
    }
    return total;
}

/* Width of the positional code of x: u itself plus a sine and a cosine
 * per axis and band. */
int orc_pos_dim(const orc_config *c)
{
    return c->pos_bands > 0 ? 3 + 6 * c->pos_bands : 0;
}

int orc_input_dim(const orc_config *c)
{
    return c->n_levels * c->n_features + orc_pos_dim(c) + c->sh_bands * c->sh_bands
           + c->n_extra * 2 * c->extra_bands;
}

/* Parameter layout: [grid entries x F][W_0][W_1]..[W_H], each W row-major
 * [out][in]; W_0: width x in, hidden: width x width, last: n_out x width.
 * No biases (the paper names none). */
int64_t orc_n_params(const orc_config *c)
{
    int64_t g = orc_level_table(c, 0, 0, 0, 0) * c->n_features;
    int64_t in = orc_input_dim(c);
    return g + (int64_t)c->width * in
           + (int64_t)(c->n_hidden - 1) * c->width * c->width
           + (int64_t)c->n_out * c->width;
}

int64_t orc_n_grid_values(const orc_config *c)
{
    return orc_level_table(c, 0, 0, 0, 0) * c->n_features;
}

/* ------------------------------------------------------------------ */
/* Encoding: cell lookup, corner index, trilinear interpolation          */
/* ------------------------------------------------------------------ */

/* Spatial hash of the cited multi-resolution hash encoding: XOR of the
 * integer corner coordinates times the primes 1, 2654435761, 805459861,
 * wrapped to 32 bits, reduced modulo T (a power of two). */
uint32_t orc_hash(uint32_t x, uint32_t y, uint32_t z, int log2_T)
{
    uint32_t h = (x * 1u) ^ (y * 2654435761u) ^ (z * 805459861u);
    return h & (uint32_t)(((uint64_t)1 << log2_T) - 1u);
}

/* Dense index, x fastest. */
int64_t orc_dense_index(int64_t x, int64_t y, int64_t z, int64_t N)
{
    return x + (N + 1) * (y + (N + 1) * z);
}

/* Position normalisation reading: the per-axis affine map of the caller's
 * bounding box onto the level's lattice, s = p*k - a_min*k with
 * k = N / (a_max - a_min), evaluated in double with one fused rounding.
 * p is first clamped to the box.  Cell i = min(max(floor(s),0), N-1),
 * fraction f = s - i.  Returns 1 if p was outside the box. */
int orc_cell(const orc_config *c, int64_t N, const double p[3], int64_t i[3],
             double f[3])
{
    int out = 0;
    for (int a = 0; a < 3; ++a) {
        double lo = c->aabb_min[a], hi = c->aabb_max[a];
        double pc = p[a];
        if (pc < lo) { pc = lo; out = 1; }
        if (pc > hi) { pc = hi; out = 1; }
        double k = (double)N / (hi - lo);
        double s = fma(pc, k, -(lo * k));
        double fl = floor(s);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(N - 1)) fl = (double)(N - 1);
        i[a] = (int64_t)fl;
        f[a] = s - fl;
    }
    return out;
}

/* Corner c = cx + 2cy + 4cz of the cell: table index (within the level)
 * and trilinear weight. */
void orc_corner(const orc_config *c, int64_t N, int dense, const int64_t i[3],
                const double f[3], int corner, int64_t *idx, double *w)
{
    int64_t v[3];
    double wt = 1.0;
    for (int a = 0; a < 3; ++a) {
        int bit = (corner >> a) & 1;
        v[a] = i[a] + bit;
        wt *= bit ? f[a] : (1.0 - f[a]);
    }
    if (dense)
        *idx = orc_dense_index(v[0], v[1], v[2], N);
    else
        *idx = (int64_t)orc_hash((uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2],
                                 c->log2_T);
    *w = wt;
}

/* ------------------------------------------------------------------ */
/* Direction encoding: real spherical harmonics                         */
/* ------------------------------------------------------------------ */
/* Reading (the paper is silent on the direction encoding): real, orthonormal
 * SH of the unit normal with the Condon-Shortley phase, index l^2 + l + m,
 * theta measured from +z, phi = atan2(y, x).  Computed from the associated
 * Legendre recurrence. */
static double orc_factorial(int n)
{
    double r = 1.0;
    for (int k = 2; k <= n; ++k) r *= k;
    return r;
}

/* P_l^m(x) with the Condon-Shortley phase, m >= 0. */
double orc_legendre(int l, int m, double x)
{
    double pmm = 1.0;
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    for (int k = 1; k <= m; ++k) pmm *= -(2.0 * k - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

void orc_sh(int bands, const double n_unit[3], double *out)
{
    double z = n_unit[2];
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    double phi = atan2(n_unit[1], n_unit[0]);
    for (int l = 0; l < bands; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI)
                            * orc_factorial(l - am) / orc_factorial(l + am));
            double P = orc_legendre(l, am, z);
            double y;
            if (m > 0) y = sqrt(2.0) * K * cos(m * phi) * P;
            else if (m < 0) y = sqrt(2.0) * K * sin(am * phi) * P;
            else y = K * P;
            out[l * l + l + m] = y;
        }
    }
}

/* Frequency encoding of a scalar (Sec. 4.1 and Sec. 6, cited positional
 * encoding): [sin(2^k pi t), cos(2^k pi t)] for k < bands, interleaved. */
void orc_freq(int bands, double t, double *out)
{
    for (int k = 0; k < bands; ++k) {
        double a = ldexp(ORC_PI, k) * t;
        out[2 * k] = sin(a);
        out[2 * k + 1] = cos(a);
    }
}

/* ------------------------------------------------------------------ */
/* One query: encoding + MLP                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t res[64];
    int dense[64];
    int64_t size[64];
    int64_t offset[64];
    int64_t n_entries;
} orc_levels;

static void orc_levels_init(const orc_config *c, orc_levels *lv)
{
    lv->n_entries = orc_level_table(c, lv->res, lv->dense, lv->size, lv->offset);
}

/* Flags returned per query. */
#define ORC_FLAG_OUTSIDE 1   /* position outside the box (clamped) */
#define ORC_FLAG_BAD_INPUT 2 /* non-finite position/normal or zero normal */
#define ORC_FLAG_BAD_OUTPUT 4 /* non-finite output */
#define ORC_FLAG_NEG_OUTPUT 16 /* finite output with a negative channel */

/* Positional code of x for the models without grid levels (Sec. 4.1: the
 * smaller networks of Table 1 feed the position through the cited frequency
 * encoding, eight bands).  Readings: the position is first mapped onto the
 * unit cube by the box, u = (p - a_min) / (a_max - a_min), clamped as for the
 * grid; the code is u itself followed, band by band (k = 0 .. bands-1), by
 * sin(2^k pi u_x), sin(2^k pi u_y), sin(2^k pi u_z), then the three cosines.
 * Returns 1 if p was outside the box. */
int orc_pos_code(const orc_config *c, const double p[3], double *out)
{
    int outside = 0;
    double u[3];
    for (int a = 0; a < 3; ++a) {
        double lo = c->aabb_min[a], hi = c->aabb_max[a], pc = p[a];
        if (pc < lo) { pc = lo; outside = 1; }
        if (pc > hi) { pc = hi; outside = 1; }
        u[a] = (pc - lo) / (hi - lo);
        out[a] = u[a];
    }
    for (int k = 0; k < c->pos_bands; ++k)
        for (int a = 0; a < 3; ++a) {
            double ang = ldexp(ORC_PI, k) * u[a];
            out[3 + 6 * k + a] = sin(ang);
            out[3 + 6 * k + 3 + a] = cos(ang);
        }
    return outside;
}

/* Input vector x0 = concat(grid features level 0..L-1, positional code,
 * SH, freq(extra)). */
static int orc_encode(const orc_config *c, const orc_levels *lv,
                      const double *grid, const double p[3], const double n[3],
                      const double *extra, double *x0)
{
    int flags = 0;
    int F = c->n_features;
    for (int l = 0; l < c->n_levels; ++l) {
        int64_t i[3];
        double f[3];
        flags |= orc_cell(c, lv->res[l], p, i, f) ? ORC_FLAG_OUTSIDE : 0;
        for (int j = 0; j < F; ++j) x0[l * F + j] = 0.0;
        for (int corner = 0; corner < 8; ++corner) {
            int64_t idx;
            double w;
            orc_corner(c, lv->res[l], lv->dense[l], i, f, corner, &idx, &w);
            const double *e = grid + (lv->offset[l] + idx) * F;
            for (int j = 0; j < F; ++j) x0[l * F + j] += w * e[j];
        }
    }
    int k = c->n_levels * F;
    if (c->pos_bands > 0) {
        flags |= orc_pos_code(c, p, x0 + k) ? ORC_FLAG_OUTSIDE : 0;
        k += orc_pos_dim(c);
    }
    if (c->sh_bands > 0) {
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double u[3] = {n[0] / len, n[1] / len, n[2] / len};
        orc_sh(c->sh_bands, u, x0 + k);
        k += c->sh_bands * c->sh_bands;
    }
    for (int e = 0; e < c->n_extra; ++e) {
        orc_freq(c->extra_bands, extra[e], x0 + k);
        k += 2 * c->extra_bands;
    }
    return flags;
}

/* Pointers to the weight matrices inside a flat parameter vector. */
static void orc_weight_ptrs(const orc_config *c, const double *params,
                            const double **W)
{
    const double *w = params + orc_n_grid_values(c);
    int in = orc_input_dim(c);
    W[0] = w;
    w += (int64_t)c->width * in;
    for (int h = 1; h < c->n_hidden; ++h) {
        W[h] = w;
        w += (int64_t)c->width * c->width;
    }
    W[c->n_hidden] = w;
}

/* Forward through the MLP (Sec. 4.1): x_{k+1} = max(0, W_k x_k) for the
 * hidden layers, E = W_H x_H.  If `acts` is given it receives x_0 .. x_H
 * (post-activation) concatenated. */
static void orc_mlp(const orc_config *c, const double *const *W, const double *x0,
                    double *out, double *acts)
{
    int in = orc_input_dim(c);
    double bufA[1024], bufB[1024];
    const double *x = x0;
    int xd = in;
    double *y = bufA;
    if (acts) memcpy(acts, x0, sizeof(double) * in);
    double *ap = acts ? acts + in : 0;
    for (int h = 0; h < c->n_hidden; ++h) {
        const double *Wh = W[h];
        for (int o = 0; o < c->width; ++o) {
            double s = 0.0;
            for (int q = 0; q < xd; ++q) s += Wh[(int64_t)o * xd + q] * x[q];
            y[o] = s > 0.0 ? s : 0.0;
        }
        if (ap) { memcpy(ap, y, sizeof(double) * c->width); ap += c->width; }
        x = y;
        xd = c->width;
        y = (y == bufA) ? bufB : bufA;
    }
    const double *WH = W[c->n_hidden];
    for (int o = 0; o < c->n_out; ++o) {
        double s = 0.0;
        for (int q = 0; q < xd; ++q) s += WH[(int64_t)o * xd + q] * x[q];
        out[o] = s;
    }
}

/* Batch query (Sec. 4.4 rendering): for every point with mask != 0 compute
 * E = E_theta(x, n[, extra]) and L = albedo * E / pi (Eq. 2).  Points with
 * mask == 0 get E = L = 0 and no flags; a degenerate input (non-finite
 * value, zero normal) gets E = L = 0 and the bad-input flag.  `extra` is per point
 * ([count][n_extra]) or NULL when n_extra == 0.  Any of albedo, mask,
 * out_L, out_flags may be NULL. */
void orc_query(const orc_config *c, const double *params, int64_t count,
               const float *pos, const float *nrm, const float *extra,
               const float *albedo, const uint8_t *mask, double *out_E,
               double *out_L, uint8_t *out_flags, double *out_x0)
{
    orc_levels lv;
    orc_levels_init(c, &lv);
    const double *W[64];
    orc_weight_ptrs(c, params, W);
    int in = orc_input_dim(c);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < count; ++q) {
        double x0[1024], E[16], ex[8];
        double p[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
        double n[3] = {nrm[3 * q], nrm[3 * q + 1], nrm[3 * q + 2]};
        int flags = 0;
        int bad = 0;
        int on = mask ? mask[q] != 0 : 1;
        for (int a = 0; a < 3; ++a) bad |= !isfinite(p[a]) || !isfinite(n[a]);
        if (!bad && c->sh_bands > 0 && n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0)
            bad = 1;
        for (int e = 0; e < c->n_extra; ++e) {
            ex[e] = extra ? extra[q * c->n_extra + e] : 0.0;
            bad |= !isfinite(ex[e]);
        }
        for (int o = 0; o < c->n_out; ++o) E[o] = 0.0;
        if (on && bad) flags |= ORC_FLAG_BAD_INPUT;
        if (on && !bad) {
            flags |= orc_encode(c, &lv, params, p, n, ex, x0);
            if (out_x0) memcpy(out_x0 + q * in, x0, sizeof(double) * in);
            orc_mlp(c, W, x0, E, 0);
            int neg = 0;
            for (int o = 0; o < c->n_out; ++o) {
                if (!isfinite(E[o])) flags |= ORC_FLAG_BAD_OUTPUT;
                neg |= E[o] < 0.0;
            }
            /* irradiance is non-negative; the linear output layer is not */
            if (neg && !(flags & ORC_FLAG_BAD_OUTPUT)) flags |= ORC_FLAG_NEG_OUTPUT;
        }
        for (int o = 0; o < c->n_out; ++o) {
            out_E[q * c->n_out + o] = E[o];
            if (out_L) {
                double rho = albedo ? albedo[3 * q + (o < 3 ? o : 2)] : 1.0;
                out_L[q * c->n_out + o] = rho * E[o] / ORC_PI;
            }
        }
        if (out_flags) out_flags[q] = (uint8_t)flags;
    }
}

/* Corner indices and weights of one point at every level (for the exact
 * integer check).  idx: [L][8] within-level indices; w: [L][8]. */
void orc_corners(const orc_config *c, const float *pos, int64_t *idx, double *w)
{
    orc_levels lv;
    orc_levels_init(c, &lv);
    double p[3] = {pos[0], pos[1], pos[2]};
    for (int l = 0; l < c->n_levels; ++l) {
        int64_t i[3];
        double f[3];
        orc_cell(c, lv.res[l], p, i, f);
        for (int k = 0; k < 8; ++k)
            orc_corner(c, lv.res[l], lv.dense[l], i, f, k, idx + l * 8 + k, w + l * 8 + k);
    }
}

/* orc_corners for n points: idx [n][L][8] within-level indices. */
void orc_corners_n(const orc_config *c, const float *pos, int64_t n, int64_t *idx)
{
#pragma omp parallel
    {
        double *w = (double *)malloc(sizeof(double) * 8 * (size_t)(c->n_levels > 0 ? c->n_levels : 1));
#pragma omp for schedule(static)
        for (int64_t q = 0; q < n; ++q)
            orc_corners(c, pos + 3 * q, idx + q * c->n_levels * 8, w);
        free(w);
    }
}

/* ------------------------------------------------------------------ */
/* Training: Eq. 3 loss, exact backpropagation, Adam                     */
/* ------------------------------------------------------------------ */
/* Relative L2 (Eq. 3): per sample and channel (E_hat - E)^2 / (sg(E_hat^2)
 * + eps), eps = 0.01.  Reading: mean over the `count` samples and the n_out
 * channels; samples with valid == 0 contribute nothing (but stay in the
 * count).  grads (same layout as params) receives d loss / d params,
 * accumulated over the batch.  Returns the loss. */
double orc_loss_grad(const orc_config *c, const double *params, int64_t count,
                     const float *pos, const float *nrm, const float *extra,
                     const float *target, const uint8_t *valid, double eps,
                     double *grads)
{
    orc_levels lv;
    orc_levels_init(c, &lv);
    const double *W[64];
    orc_weight_ptrs(c, params, W);
    int in = orc_input_dim(c), H = c->n_hidden, Wd = c->width, F = c->n_features;
    int64_t np_ = orc_n_params(c);
    memset(grads, 0, sizeof(double) * np_);
    double *gW0 = grads + orc_n_grid_values(c);
    double loss = 0.0;
    double inv = 1.0 / ((double)count * c->n_out);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nthreads * np_, sizeof(double));
    double *lossp = (double *)calloc((size_t)nthreads, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = priv + (size_t)tid * np_;
        double *gW = g + orc_n_grid_values(c);
        double x0[1024], acts[8192], dE[16], d[1024], dn[1024], ex[8];
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < count; ++q) {
            if (valid && !valid[q]) continue;
            double p[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
            double n[3] = {nrm[3 * q], nrm[3 * q + 1], nrm[3 * q + 2]};
            for (int e = 0; e < c->n_extra; ++e) ex[e] = extra ? extra[q * c->n_extra + e] : 0.0;
            orc_encode(c, &lv, params, p, n, ex, x0);
            double E[16];
            orc_mlp(c, W, x0, E, acts);
            for (int o = 0; o < c->n_out; ++o) {
                double y = target[q * c->n_out + o];
                double den = E[o] * E[o] + eps; /* held constant: stop-gradient */
                double r = E[o] - y;
                lossp[tid] += r * r / den * inv;
                dE[o] = 2.0 * r / den * inv;
            }
            /* acts layout: x_0 (in), x_1 .. x_H (width each). */
            const double *xH = acts + in + (int64_t)(H - 1) * Wd;
            double *gWH = gW + (int64_t)Wd * in + (int64_t)(H - 1) * Wd * Wd;
            for (int o = 0; o < c->n_out; ++o)
                for (int k = 0; k < Wd; ++k) gWH[(int64_t)o * Wd + k] += dE[o] * xH[k];
            for (int k = 0; k < Wd; ++k) {
                double s = 0.0;
                for (int o = 0; o < c->n_out; ++o) s += W[H][(int64_t)o * Wd + k] * dE[o];
                d[k] = s; /* gradient w.r.t. x_H */
            }
            for (int h = H - 1; h >= 0; --h) {
                const double *xo = acts + in + (int64_t)h * Wd;        /* x_{h+1} */
                const double *xi = h == 0 ? acts : acts + in + (int64_t)(h - 1) * Wd;
                int di = h == 0 ? in : Wd;
                /* through ReLU: x_{h+1} = max(0, z); derivative 1 where z > 0,
                 * i.e. where x_{h+1} > 0 (ReLU'(0) = 0). */
                for (int k = 0; k < Wd; ++k) d[k] = xo[k] > 0.0 ? d[k] : 0.0;
                double *gWh = h == 0 ? gW : gW + (int64_t)Wd * in + (int64_t)(h - 1) * Wd * Wd;
                for (int o = 0; o < Wd; ++o)
                    for (int k = 0; k < di; ++k) gWh[(int64_t)o * di + k] += d[o] * xi[k];
                for (int k = 0; k < di; ++k) {
                    double s = 0.0;
                    for (int o = 0; o < Wd; ++o) s += W[h][(int64_t)o * di + k] * d[o];
                    dn[k] = s;
                }
                memcpy(d, dn, sizeof(double) * di);
            }
            /* d now holds d loss / d x_0; scatter the grid part to the corners. */
            for (int l = 0; l < c->n_levels; ++l) {
                int64_t i[3];
                double f[3];
                orc_cell(c, lv.res[l], p, i, f);
                for (int corner = 0; corner < 8; ++corner) {
                    int64_t idx;
                    double w;
                    orc_corner(c, lv.res[l], lv.dense[l], i, f, corner, &idx, &w);
                    double *ge = g + (lv.offset[l] + idx) * F;
                    for (int j = 0; j < F; ++j) ge[j] += w * d[l * F + j];
                }
            }
        }
    }
    for (int t = 0; t < nthreads; ++t) {
        const double *g = priv + (size_t)t * np_;
        for (int64_t k = 0; k < np_; ++k) grads[k] += g[k];
        loss += lossp[t];
    }
    (void)gW0;
    free(priv);
    free(lossp);
    return loss;
}

/* Loss only (for finite differences). */
double orc_loss(const orc_config *c, const double *params, int64_t count,
                const float *pos, const float *nrm, const float *extra,
                const float *target, const uint8_t *valid, double eps)
{
    orc_levels lv;
    orc_levels_init(c, &lv);
    const double *W[64];
    orc_weight_ptrs(c, params, W);
    double loss = 0.0;
    double inv = 1.0 / ((double)count * c->n_out);
    for (int64_t q = 0; q < count; ++q) {
        if (valid && !valid[q]) continue;
        double x0[1024], E[16], ex[8];
        double p[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
        double n[3] = {nrm[3 * q], nrm[3 * q + 1], nrm[3 * q + 2]};
        for (int e = 0; e < c->n_extra; ++e) ex[e] = extra ? extra[q * c->n_extra + e] : 0.0;
        orc_encode(c, &lv, params, p, n, ex, x0);
        orc_mlp(c, W, x0, E, 0);
        for (int o = 0; o < c->n_out; ++o) {
            double r = E[o] - target[q * c->n_out + o];
            loss += r * r / (E[o] * E[o] + eps) * inv;
        }
    }
    return loss;
}

/* Adam (Kingma & Ba, Algorithm 1), applied densely to every parameter;
 * `step` is the 1-based iteration t. */
void orc_adam(int64_t n, double *params, const double *grads, double *m, double *v,
              double lr, double beta1, double beta2, double eps, int64_t step)
{
    double bc1 = 1.0 - pow(beta1, (double)step);
    double bc2 = 1.0 - pow(beta2, (double)step);
    for (int64_t k = 0; k < n; ++k) {
        double g = grads[k];
        m[k] = beta1 * m[k] + (1.0 - beta1) * g;
        v[k] = beta2 * v[k] + (1.0 - beta2) * g * g;
        double mh = m[k] / bc1, vh = v[k] / bc2;
        params[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Learning rate schedule (Sec. 4.5): lr0 until step s1, then exponential
 * decay reaching lr1 at step s_end (reading: decay ends at the last step). */
double orc_lr(int64_t step, int64_t s1, int64_t s_end, double lr0, double lr1)
{
    if (step <= s1 || s_end <= s1) return lr0;
    double t = (double)(step - s1) / (double)(s_end - s1);
    if (t > 1.0) t = 1.0;
    return lr0 * pow(lr1 / lr0, t);
}

/* ------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x64-10                           */
/* ------------------------------------------------------------------ */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11): ten rounds of two 64x64->128 multiplies with the published
 * multipliers and Weyl key increments. */
static void orc_mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    __uint128_t p = (__uint128_t)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        orc_mulhilo64(M0, x0, &h0, &l0);
        orc_mulhilo64(M1, x2, &h1, &l1);
        uint64_t y0 = h1 ^ x1 ^ k0, y1 = l1, y2 = h0 ^ x3 ^ k1, y3 = l0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform number `dim` of the stream (seed, a, b, stream): block dim/8 of
 * Philox with counter (a, b, block, stream) and key (seed, 0); 32-bit half
 * dim%2 (low first) of word (dim%8)/2, mapped to [0,1) with 24 bits. */
double orc_uniform(uint64_t seed, uint64_t a, uint64_t b, uint64_t stream, int dim)
{
    uint64_t ctr[4] = {a, b, (uint64_t)(dim / 8), stream}, key[2] = {seed, 0};
    uint64_t out[4];
    orc_philox4x64(ctr, key, out);
    int w = (dim % 8) / 2;
    uint32_t u = (dim & 1) ? (uint32_t)(out[w] >> 32) : (uint32_t)out[w];
    return (double)(u >> 8) * 0x1p-24;
}

/* Seeded initial parameters.  The paper does not state its initialisation;
 * reading: grid values uniform on [lo, hi) (the cited hash encoding starts
 * its table near zero), weights Xavier-uniform (Glorot and Bengio, 2010):
 * uniform on [-a, a) with a = sqrt(6 / (fan_in + fan_out)) per matrix.
 * Parameter k draws uniform number 0 of generator stream (seed, k, 0, 3);
 * the value is formed in double precision and rounded once to float. */
void orc_init_params(const orc_config *c, uint64_t seed, double lo, double hi, float *out)
{
    int64_t n_grid = orc_n_grid_values(c);
    int64_t n = orc_n_params(c);
    int n_mats = c->n_hidden + 1;
    int64_t k = 0;
    for (; k < n_grid; ++k) {
        double u = orc_uniform(seed, (uint64_t)k, 0, 3, 0);
        out[k] = (float)fma(hi - lo, u, lo);
    }
    for (int m = 0; m < n_mats; ++m) {
        int64_t fan_in = m == 0 ? orc_input_dim(c) : c->width;
        int64_t fan_out = m == n_mats - 1 ? c->n_out : c->width;
        double a = sqrt(6.0 / (double)(fan_in + fan_out));
        for (int64_t e = 0; e < fan_in * fan_out; ++e, ++k) {
            double u = orc_uniform(seed, (uint64_t)k, 0, 3, 0);
            double t = 2.0 * u;
            t = t - 1.0;
            out[k] = (float)(a * t);
        }
    }
    (void)n;
}

/* ------------------------------------------------------------------ */
/* Scenes and ray casting                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t kind;       /* 0 box, 1 rect, 2 disk */
    int32_t axis;
    float sign;
    float p[3];
    float q[3];
    float radius;
    float albedo[3];
    float emission[3];
} orc_prim;

typedef struct {
    double t;
    int prim;
    double nrm[3];      /* geometric normal of the front side of the surface */
    int back;           /* hit from behind */
} orc_hit;

static int orc_is_light(const orc_prim *pr)
{
    return pr->emission[0] > 0.f || pr->emission[1] > 0.f || pr->emission[2] > 0.f;
}

/* Closest hit with t > tmin; ties go to the lowest primitive index.
 * shift (or NULL): primitive k is translated by shift[3k..3k+2]; it is
 * tested with the ray origin moved by the opposite amount, which gives the
 * same distance, side and normal. */
static int orc_trace_at(const orc_prim *prims, int n, const double o_in[3],
                        const double d[3], double tmin, orc_hit *h, const double *shift)
{
    h->t = INFINITY;
    h->prim = -1;
    for (int k = 0; k < n; ++k) {
        const orc_prim *pr = &prims[k];
        double o[3] = {o_in[0], o_in[1], o_in[2]};
        if (shift)
            for (int a = 0; a < 3; ++a) o[a] -= shift[3 * k + a];
        if (pr->kind == 0) {
            double tn = -INFINITY, tf = INFINITY;
            int an = -1, af = -1, miss = 0;
            for (int a = 0; a < 3; ++a) {
                double lo = pr->p[a], hi = pr->q[a];
                if (d[a] == 0.0) {
                    if (o[a] < lo || o[a] > hi) { miss = 1; break; }
                    continue;
                }
                double t1 = (lo - o[a]) / d[a], t2 = (hi - o[a]) / d[a];
                double ta = t1 < t2 ? t1 : t2, tb = t1 < t2 ? t2 : t1;
                if (ta > tn) { tn = ta; an = a; }
                if (tb < tf) { tf = tb; af = a; }
            }
            if (miss || tn > tf) continue;
            if (tn > tmin && an >= 0) {
                if (tn < h->t) {
                    h->t = tn; h->prim = k; h->back = 0;
                    h->nrm[0] = h->nrm[1] = h->nrm[2] = 0.0;
                    h->nrm[an] = d[an] > 0 ? -1.0 : 1.0;
                }
            } else if (tf > tmin && af >= 0) {
                if (tf < h->t) {
                    h->t = tf; h->prim = k; h->back = 1;
                    h->nrm[0] = h->nrm[1] = h->nrm[2] = 0.0;
                    h->nrm[af] = d[af] > 0 ? 1.0 : -1.0; /* outward normal of the exit face */
                }
            }
        } else if (pr->kind == 1) {
            int a = pr->axis, u = (a + 1) % 3, v = (a + 2) % 3;
            if (d[a] == 0.0) continue;
            double t = (pr->p[a] - o[a]) / d[a];
            if (!(t > tmin) || !(t < h->t)) continue;
            double hu = o[u] + t * d[u], hv = o[v] + t * d[v];
            if (fabs(hu - pr->p[u]) > pr->q[0] || fabs(hv - pr->p[v]) > pr->q[1]) continue;
            h->t = t; h->prim = k;
            h->nrm[0] = h->nrm[1] = h->nrm[2] = 0.0;
            h->nrm[a] = pr->sign;
            h->back = d[a] * pr->sign > 0.0;
        } else {
            double nn[3] = {pr->q[0], pr->q[1], pr->q[2]};
            double den = d[0] * nn[0] + d[1] * nn[1] + d[2] * nn[2];
            if (den == 0.0) continue;
            double t = ((pr->p[0] - o[0]) * nn[0] + (pr->p[1] - o[1]) * nn[1]
                        + (pr->p[2] - o[2]) * nn[2]) / den;
            if (!(t > tmin) || !(t < h->t)) continue;
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double e = o[a] + t * d[a] - pr->p[a];
                r2 += e * e;
            }
            if (r2 > (double)pr->radius * pr->radius) continue;
            h->t = t; h->prim = k;
            for (int a = 0; a < 3; ++a) h->nrm[a] = nn[a];
            h->back = den > 0.0;
        }
    }
    return h->prim >= 0;
}

static int orc_trace(const orc_prim *prims, int n, const double o[3],
                     const double d[3], double tmin, orc_hit *h)
{
    return orc_trace_at(prims, n, o, d, tmin, h, 0);
}

/* Orthonormal basis around a unit vector (Duff et al., "Building an
 * Orthonormal Basis, Revisited", JCGT 2017). */
static void orc_onb(const double n[3], double t[3], double b[3])
{
    double s = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double bb = n[0] * n[1] * a;
    t[0] = 1.0 + s * n[0] * n[0] * a; t[1] = s * bb; t[2] = -s * n[0];
    b[0] = bb; b[1] = s + n[1] * n[1] * a; b[2] = -n[1];
}

/* Cosine-distributed direction about n (Malley's method): a uniform point
 * on the unit disk, r = sqrt(u1), phi = 2 pi u2, lifted to the hemisphere. */
static void orc_cosine_dir(const double n[3], double u1, double u2, double d[3])
{
    double t[3], b[3];
    orc_onb(n, t, b);
    double r = sqrt(u1), phi = 2.0 * ORC_PI * u2;
    double x = r * cos(phi), y = r * sin(phi), z = sqrt(fmax(0.0, 1.0 - u1));
    for (int a = 0; a < 3; ++a) d[a] = x * t[a] + y * b[a] + z * n[a];
}

/* Uniform point on a light's front surface; returns its area. */
static double orc_light_point(const orc_prim *pr, double u1, double u2, double q[3],
                              double nq[3])
{
    if (pr->kind == 1) {
        int a = pr->axis, u = (a + 1) % 3, v = (a + 2) % 3;
        q[a] = pr->p[a];
        q[u] = pr->p[u] + (2.0 * u1 - 1.0) * pr->q[0];
        q[v] = pr->p[v] + (2.0 * u2 - 1.0) * pr->q[1];
        nq[0] = nq[1] = nq[2] = 0.0;
        nq[a] = pr->sign;
        return 4.0 * (double)pr->q[0] * pr->q[1];
    } else if (pr->kind == 2) {
        double n[3] = {pr->q[0], pr->q[1], pr->q[2]}, t[3], b[3];
        orc_onb(n, t, b);
        double r = pr->radius * sqrt(u1), phi = 2.0 * ORC_PI * u2;
        for (int a = 0; a < 3; ++a) {
            q[a] = pr->p[a] + r * (cos(phi) * t[a] + sin(phi) * b[a]);
            nq[a] = n[a];
        }
        return ORC_PI * (double)pr->radius * pr->radius;
    }
    return 0.0;
}

#define ORC_MC_NEE 1
#define ORC_MC_EMIT_ON_HIT 2
#define ORC_MC_INCLUDE_DIRECT 4
#define ORC_MC_DIRECT_AT_ORIGIN 8

/* Monte Carlo estimate of E(x, n), Eq. 1, restricted to indirect light
 * (Sec. 3): light that left an emitter and was reflected 1..B times before
 * reaching x.  Per sample: a cosine-distributed direction about n (so the
 * estimator is pi times the radiance found along it); at the first hit y_1,
 * emission is direct and skipped (unless INCLUDE_DIRECT); a hit from behind
 * is counted and scores 0 (culling, Sec. 4.5); then for k = 1..B the
 * radiance reflected at y_k is gathered by next-event estimation to every
 * light (NEE) or by emission found by the continuation ray (EMIT_ON_HIT),
 * and the path continues with a cosine-sampled direction and throughput
 * times albedo.  DIRECT_AT_ORIGIN replaces all of this by light sampling of
 * the direct irradiance at x itself (a test mode).
 * The random stream of point i is keyed by point_id[i] (i when point_id is
 * NULL).  Random dimensions of sample s: 0-1 first direction; bounce k
 * (1-based) uses 2 + (k-1)(2J+2) + 2j for light j and 2 + (k-1)(2J+2) + 2J
 * for the continuation, J = number of lights.  DIRECT_AT_ORIGIN uses 2j.
 * Outputs per point: mean E (3), variance of the mean (3), back-face count,
 * valid = (back-face count <= S/2) and some channel of E > 0.
 * A scene that changes with a scene variable (Sec. 6: moving emitters or
 * occluders): motion [n_prims][3] (or NULL) and tvar [count] (or NULL, t =
 * 0); at point i primitive k occupies its place translated by
 * tvar[i] * motion[k].  The ray offset eps uses the scene's extent at t = 0. */
void orc_mc_irradiance(const orc_prim *prims, int n_prims, const float *x,
                       const float *nrm, const uint64_t *point_id, int64_t count, int spp,
                       int bounces, int flags, uint64_t seed, double *out_E, double *out_var,
                       int32_t *out_backfaces, uint8_t *out_valid, const float *motion,
                       const float *tvar)
{
    int lights[64], J = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < n_prims; ++k) {
        const orc_prim *pr = &prims[k];
        if (orc_is_light(pr) && J < 64) lights[J++] = k;
        double a[3], b[3];
        if (pr->kind == 0) {
            for (int c = 0; c < 3; ++c) { a[c] = pr->p[c]; b[c] = pr->q[c]; }
        } else if (pr->kind == 1) {
            int ax = pr->axis, u = (ax + 1) % 3, v = (ax + 2) % 3;
            for (int c = 0; c < 3; ++c) a[c] = b[c] = pr->p[c];
            a[u] -= pr->q[0]; b[u] += pr->q[0]; a[v] -= pr->q[1]; b[v] += pr->q[1];
        } else {
            for (int c = 0; c < 3; ++c) { a[c] = pr->p[c] - pr->radius; b[c] = pr->p[c] + pr->radius; }
        }
        for (int c = 0; c < 3; ++c) {
            if (a[c] < lo[c]) lo[c] = a[c];
            if (b[c] > hi[c]) hi[c] = b[c];
        }
    }
    double extent = 0.0;
    for (int c = 0; c < 3; ++c) if (hi[c] - lo[c] > extent) extent = hi[c] - lo[c];
    double eps = 1e-4 * extent;
    int stride = 2 * J + 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < count; ++i) {
        const uint64_t pid = point_id ? point_id[i] : (uint64_t)i;
        double *shift = 0;
        if (motion) {
            const double tv = tvar ? (double)tvar[i] : 0.0;
            shift = (double *)malloc(sizeof(double) * 3 * (size_t)n_prims);
            for (int k = 0; k < 3 * n_prims; ++k) shift[k] = tv * (double)motion[k];
        }
        double sum[3] = {0, 0, 0}, sum2[3] = {0, 0, 0};
        int backs = 0;
        double px[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        double pn[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        double ln = sqrt(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
        for (int a = 0; a < 3; ++a) pn[a] /= ln;
        for (int s = 0; s < spp; ++s) {
            double val[3] = {0, 0, 0};
            if (flags & ORC_MC_DIRECT_AT_ORIGIN) {
                double o[3];
                for (int a = 0; a < 3; ++a) o[a] = px[a] + eps * pn[a];
                for (int j = 0; j < J; ++j) {
                    const orc_prim *L = &prims[lights[j]];
                    double q[3], nq[3];
                    double A = orc_light_point(L, orc_uniform(seed, pid, s, 0, 2 * j),
                                               orc_uniform(seed, pid, s, 0, 2 * j + 1), q, nq);
                    if (shift) for (int a = 0; a < 3; ++a) q[a] += shift[3 * lights[j] + a];
                    double w[3] = {q[0] - o[0], q[1] - o[1], q[2] - o[2]};
                    double d2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], dl = sqrt(d2);
                    for (int a = 0; a < 3; ++a) w[a] /= dl;
                    double cy = pn[0] * w[0] + pn[1] * w[1] + pn[2] * w[2];
                    double cq = -(nq[0] * w[0] + nq[1] * w[1] + nq[2] * w[2]);
                    if (cy <= 0.0 || cq <= 0.0) continue;
                    orc_hit hh;
                    if (!orc_trace_at(prims, n_prims, o, w, 0.0, &hh, shift) || hh.prim != lights[j]) continue;
                    for (int c = 0; c < 3; ++c) val[c] += L->emission[c] * cy * cq / d2 * A;
                }
            } else {
                double o[3], d[3];
                for (int a = 0; a < 3; ++a) o[a] = px[a] + eps * pn[a];
                orc_cosine_dir(pn, orc_uniform(seed, pid, s, 0, 0),
                               orc_uniform(seed, pid, s, 0, 1), d);
                orc_hit h;
                int ok = orc_trace_at(prims, n_prims, o, d, 0.0, &h, shift);
                if (ok && h.back) { backs++; ok = 0; }
                if (ok) {
                    const orc_prim *pr = &prims[h.prim];
                    double rad[3] = {0, 0, 0};
                    if (flags & ORC_MC_INCLUDE_DIRECT)
                        for (int c = 0; c < 3; ++c) rad[c] += pr->emission[c];
                    double beta[3] = {1, 1, 1};
                    double y[3], ny[3];
                    for (int a = 0; a < 3; ++a) { y[a] = o[a] + h.t * d[a]; ny[a] = h.nrm[a]; }
                    for (int k = 1; k <= bounces; ++k) {
                        const orc_prim *py = &prims[h.prim];
                        double rho[3] = {py->albedo[0], py->albedo[1], py->albedo[2]};
                        int base = 2 + (k - 1) * stride;
                        double oy[3];
                        for (int a = 0; a < 3; ++a) oy[a] = y[a] + eps * ny[a];
                        if (flags & ORC_MC_NEE) {
                            for (int j = 0; j < J; ++j) {
                                const orc_prim *L = &prims[lights[j]];
                                double q[3], nq[3];
                                double A = orc_light_point(L, orc_uniform(seed, pid, s, 0, base + 2 * j),
                                                           orc_uniform(seed, pid, s, 0, base + 2 * j + 1), q, nq);
                                if (shift) for (int a = 0; a < 3; ++a) q[a] += shift[3 * lights[j] + a];
                                double w[3] = {q[0] - oy[0], q[1] - oy[1], q[2] - oy[2]};
                                double d2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], dl = sqrt(d2);
                                for (int a = 0; a < 3; ++a) w[a] /= dl;
                                double cy = ny[0] * w[0] + ny[1] * w[1] + ny[2] * w[2];
                                double cq = -(nq[0] * w[0] + nq[1] * w[1] + nq[2] * w[2]);
                                if (cy <= 0.0 || cq <= 0.0) continue;
                                orc_hit hh;
                                if (!orc_trace_at(prims, n_prims, oy, w, 0.0, &hh, shift) || hh.prim != lights[j])
                                    continue;
                                double G = cy * cq / d2 * A;
                                for (int c = 0; c < 3; ++c)
                                    rad[c] += beta[c] * rho[c] / ORC_PI * L->emission[c] * G;
                            }
                        }
                        int cont = (flags & ORC_MC_EMIT_ON_HIT) ? 1 : (k < bounces);
                        if (!cont) break;
                        for (int c = 0; c < 3; ++c) beta[c] *= rho[c];
                        if (beta[0] == 0.0 && beta[1] == 0.0 && beta[2] == 0.0) break;
                        orc_cosine_dir(ny, orc_uniform(seed, pid, s, 0, base + 2 * J),
                                       orc_uniform(seed, pid, s, 0, base + 2 * J + 1), d);
                        if (!orc_trace_at(prims, n_prims, oy, d, 0.0, &h, shift) || h.back) break;
                        if (flags & ORC_MC_EMIT_ON_HIT) {
                            const orc_prim *pe = &prims[h.prim];
                            for (int c = 0; c < 3; ++c) rad[c] += beta[c] * pe->emission[c];
                        }
                        for (int a = 0; a < 3; ++a) { y[a] = oy[a] + h.t * d[a]; ny[a] = h.nrm[a]; }
                    }
                    for (int c = 0; c < 3; ++c) val[c] = ORC_PI * rad[c];
                }
            }
            for (int c = 0; c < 3; ++c) { sum[c] += val[c]; sum2[c] += val[c] * val[c]; }
        }
        int any = 0;
        for (int c = 0; c < 3; ++c) {
            double mean = sum[c] / spp;
            double var = spp > 1 ? (sum2[c] - spp * mean * mean) / (spp - 1.0) / spp : 0.0;
            if (var < 0.0) var = 0.0;
            out_E[3 * i + c] = mean;
            if (out_var) out_var[3 * i + c] = var;
            any |= mean > 0.0;
        }
        if (out_backfaces) out_backfaces[i] = backs;
        if (out_valid) out_valid[i] = (uint8_t)((2 * backs <= spp) && any);
        free(shift);
    }
}

/* Training points (Sec. 4.5, App. H): the first count - n_surface points
 * are uniform in the box [lo, hi] with a direction uniform on the sphere;
 * the last n_surface points are uniform by area over the non-emitting
 * surfaces (rectangles and box faces) with n = the surface's front normal.
 * Random stream 1 of the counter-based generator, counter (i, 0, block, 1).
 * Volume point: dims 0-2 position, 3-4 direction (z = 1 - 2u, phi = 2 pi u).
 * Surface point: dim 0 picks the face through the cumulative area table,
 * dims 1-2 place the point on it.  out_t (or NULL): a scene variable per
 * point uniform on [0, 1) (Sec. 6: sampled at random for training), dim 7. */
void orc_sample_points(const orc_prim *prims, int n_prims, const double lo[3],
                       const double hi[3], int64_t count, int64_t n_surface,
                       uint64_t seed, float *out_x, float *out_n, float *out_t)
{
    /* faces: (prim, face) with area; box faces 0..5 = -x,+x,-y,+y,-z,+z */
    int64_t nf = 0;
    int *fp = (int *)malloc(sizeof(int) * (6 * (size_t)n_prims + 1));
    int *ff = (int *)malloc(sizeof(int) * (6 * (size_t)n_prims + 1));
    double *cdf = (double *)malloc(sizeof(double) * (6 * (size_t)n_prims + 1));
    double acc = 0.0;
    for (int k = 0; k < n_prims; ++k) {
        const orc_prim *pr = &prims[k];
        if (orc_is_light(pr)) continue;
        if (pr->kind == 1) {
            acc += 4.0 * (double)pr->q[0] * pr->q[1];
            fp[nf] = k; ff[nf] = -1; cdf[nf] = acc; nf++;
        } else if (pr->kind == 0) {
            for (int f = 0; f < 6; ++f) {
                int a = f / 2, u = (a + 1) % 3, v = (a + 2) % 3;
                acc += ((double)pr->q[u] - pr->p[u]) * ((double)pr->q[v] - pr->p[v]);
                fp[nf] = k; ff[nf] = f; cdf[nf] = acc; nf++;
            }
        }
    }
    for (int64_t i = 0; i < count; ++i) {
        double u0 = orc_uniform(seed, i, 0, 1, 0), u1 = orc_uniform(seed, i, 0, 1, 1),
               u2 = orc_uniform(seed, i, 0, 1, 2);
        if (i < count - n_surface) {
            double u3 = orc_uniform(seed, i, 0, 1, 3), u4 = orc_uniform(seed, i, 0, 1, 4);
            double p[3] = {lo[0] + u0 * (hi[0] - lo[0]), lo[1] + u1 * (hi[1] - lo[1]),
                           lo[2] + u2 * (hi[2] - lo[2])};
            double z = 1.0 - 2.0 * u3, phi = 2.0 * ORC_PI * u4, r = sqrt(fmax(0.0, 1.0 - z * z));
            double n[3] = {r * cos(phi), r * sin(phi), z};
            for (int a = 0; a < 3; ++a) { out_x[3 * i + a] = (float)p[a]; out_n[3 * i + a] = (float)n[a]; }
            if (out_t) out_t[i] = (float)orc_uniform(seed, (uint64_t)i, 0, 1, 7);
        } else {
            double target = u0 * acc;
            int64_t lo_i = 0, hi_i = nf - 1;
            while (lo_i < hi_i) { /* first face whose cumulative area exceeds target */
                int64_t mid = (lo_i + hi_i) / 2;
                if (cdf[mid] > target) hi_i = mid; else lo_i = mid + 1;
            }
            const orc_prim *pr = &prims[fp[lo_i]];
            double p[3], n[3] = {0, 0, 0};
            if (ff[lo_i] < 0) {
                int a = pr->axis, u = (a + 1) % 3, v = (a + 2) % 3;
                p[a] = pr->p[a];
                p[u] = pr->p[u] + (2.0 * u1 - 1.0) * pr->q[0];
                p[v] = pr->p[v] + (2.0 * u2 - 1.0) * pr->q[1];
                n[a] = pr->sign;
            } else {
                int f = ff[lo_i], a = f / 2, u = (a + 1) % 3, v = (a + 2) % 3;
                p[a] = (f & 1) ? pr->q[a] : pr->p[a];
                p[u] = pr->p[u] + u1 * ((double)pr->q[u] - pr->p[u]);
                p[v] = pr->p[v] + u2 * ((double)pr->q[v] - pr->p[v]);
                n[a] = (f & 1) ? 1.0 : -1.0;
            }
            for (int a = 0; a < 3; ++a) { out_x[3 * i + a] = (float)p[a]; out_n[3 * i + a] = (float)n[a]; }
            if (out_t) out_t[i] = (float)orc_uniform(seed, (uint64_t)i, 0, 1, 7);
        }
    }
    free(fp); free(ff); free(cdf);
}

/* ------------------------------------------------------------------ */
/* Half-resolution rendering: joint bilateral upsampling                 */
/* ------------------------------------------------------------------ */
/* Sec. 4.4 renders the network at a quarter of the pixels and multiplies by
 * the full-resolution albedo; it leaves the upsampler to the cited joint
 * bilateral method.  Readings: the half-resolution samples are the
 * G-buffer pixels (2x, 2y), x < ceil(W/2), y < ceil(H/2), whose irradiance
 * half_E [ceil(H/2)][ceil(W/2)][3] is given.  A sample is usable iff its
 * pixel is covered (mask) and its position and normal are finite with a
 * non-zero normal.  Full-resolution pixel (X, Y) averages the usable
 * samples with |2x - X| <= 2 and |2y - Y| <= 2 that face its way
 * (n . n_s > 0, unit normals), with weights
 *   exp(-(dx^2 + dy^2) / (2 sigma_px^2))      spatial, dx = 2x - X (pixels)
 *   (n . n_s)^normal_power                     normal guide
 *   exp(-|p - p_s|^2 / (2 sigma_pos^2))        position guide (world units)
 * (the G-buffer guides take the place of the guide image of the cited
 * method).  The weights are formed as exp(l - l_max) from their logarithms
 * l, which leaves the average unchanged and keeps it finite however small
 * the weights.  With no usable sample facing its way the pixel takes the
 * usable sample nearest in pixels (first in row-major order among equals)
 * and flag 32; with no usable sample in the window E = 0 and flag 64.  A
 * covered pixel with a non-finite or zero-normal input gets E = 0 and flag
 * 2; a position outside the box sets flag 1.  L = albedo * E / pi (Eq. 2)
 * at full resolution. */
static int orc_px_usable(const float *pos, const float *nrm, const uint8_t *mask, int64_t i)
{
    if (mask && !mask[i]) return 0;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(pos[3 * i + a]) || !isfinite(nrm[3 * i + a])) return 0;
    return !(nrm[3 * i] == 0.0f && nrm[3 * i + 1] == 0.0f && nrm[3 * i + 2] == 0.0f);
}

static void orc_unit(const float *v, double *u)
{
    double n = sqrt((double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2]);
    for (int a = 0; a < 3; ++a) u[a] = v[a] / n;
}

void orc_upsample(const orc_config *c, int width, int height, const float *pos,
                  const float *nrm, const uint8_t *mask, const float *albedo,
                  const double *half_E, double sigma_px, double sigma_pos, int normal_power,
                  double *out_E, double *out_L, uint8_t *out_flags)
{
    const int hw = (width + 1) / 2, hh = (height + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int Y = 0; Y < height; ++Y)
        for (int X = 0; X < width; ++X) {
            const int64_t i = (int64_t)Y * width + X;
            double E[3] = {0.0, 0.0, 0.0};
            int flags = 0;
            int on = mask ? mask[i] != 0 : 1;
            if (on && !orc_px_usable(pos, nrm, mask, i)) {
                flags |= ORC_FLAG_BAD_INPUT;
            } else if (on) {
                for (int a = 0; a < 3; ++a)
                    if (pos[3 * i + a] < c->aabb_min[a] || pos[3 * i + a] > c->aabb_max[a])
                        flags |= ORC_FLAG_OUTSIDE;
                double n[3];
                orc_unit(nrm + 3 * i, n);
                double lw[9], ev[9][3];
                int ns_ = 0;
                int64_t nearest = -1;
                int best_d2 = 1 << 30, any_sample = 0;
                for (int y = (Y - 1) / 2; y <= (Y + 2) / 2; ++y) {
                    if (y < 0 || y >= hh || 2 * y - Y < -2 || 2 * y - Y > 2) continue;
                    for (int x = (X - 1) / 2; x <= (X + 2) / 2; ++x) {
                        if (x < 0 || x >= hw || 2 * x - X < -2 || 2 * x - X > 2) continue;
                        const int64_t s = (int64_t)(2 * y) * width + 2 * x;
                        if (!orc_px_usable(pos, nrm, mask, s)) continue;
                        any_sample = 1;
                        const int dx = 2 * x - X, dy = 2 * y - Y, d2 = dx * dx + dy * dy;
                        if (d2 < best_d2) { best_d2 = d2; nearest = (int64_t)y * hw + x; }
                        double nsu[3];
                        orc_unit(nrm + 3 * s, nsu);
                        double cs = n[0] * nsu[0] + n[1] * nsu[1] + n[2] * nsu[2];
                        if (!(cs > 0.0)) continue;
                        double dp2 = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            double d = (double)pos[3 * i + a] - (double)pos[3 * s + a];
                            dp2 += d * d;
                        }
                        lw[ns_] = -(double)d2 / (2.0 * sigma_px * sigma_px) + normal_power * log(cs)
                                  - dp2 / (2.0 * sigma_pos * sigma_pos);
                        const double *e = half_E + 3 * ((int64_t)y * hw + x);
                        for (int a = 0; a < 3; ++a) ev[ns_][a] = e[a];
                        ++ns_;
                    }
                }
                if (ns_ > 0) {
                    double lmax = lw[0], wsum = 0.0, acc[3] = {0.0, 0.0, 0.0};
                    for (int k = 1; k < ns_; ++k) lmax = lw[k] > lmax ? lw[k] : lmax;
                    for (int k = 0; k < ns_; ++k) {
                        double w = exp(lw[k] - lmax);
                        wsum += w;
                        for (int a = 0; a < 3; ++a) acc[a] += w * ev[k][a];
                    }
                    for (int a = 0; a < 3; ++a) E[a] = acc[a] / wsum;
                } else if (any_sample) {
                    for (int a = 0; a < 3; ++a) E[a] = half_E[3 * nearest + a];
                    flags |= 32;
                } else {
                    flags |= 64;
                }
            }
            for (int a = 0; a < 3; ++a) {
                out_E[3 * i + a] = E[a];
                if (out_L) out_L[3 * i + a] = (albedo ? albedo[3 * i + a] : 1.0) * E[a] / ORC_PI;
            }
            if (out_flags) out_flags[i] = (uint8_t)flags;
        }
}

/* ---------------------------------------------------------------- dynamic AO
 * Dynamic ambient occlusion (Sec. 4.4): at a shading point only the dynamic
 * geometry (triangles placed at render time) is tested for obstruction of
 * the hemisphere.  Reading: the returned visibility is one minus the
 * cosine-weighted fraction of directions whose ray from x + eps n meets a
 * dynamic triangle at a distance in (0, radius]; triangles count from both
 * sides.  It is estimated with `rays` cosine-distributed directions from the
 * point's own random stream (stream 2, dimensions 0 and 1 of sample k), so
 * the estimate is a deterministic function of (seed, point id).  The shaded
 * irradiance is the model's E times this visibility. */

/* Ray-triangle test (Moller and Trumbore, 1997): barycentric (u, v) and
 * distance t from Cramer's rule on o + t d = v0 + u e1 + v e2. */
static int orc_tri_hit(const double o[3], const double d[3], const float *tri, double tmax)
{
    double v0[3], e1[3], e2[3], p[3], s[3], q[3];
    for (int a = 0; a < 3; ++a) {
        v0[a] = tri[a];
        e1[a] = (double)tri[3 + a] - v0[a];
        e2[a] = (double)tri[6 + a] - v0[a];
        s[a] = o[a] - v0[a];
    }
    p[0] = d[1] * e2[2] - d[2] * e2[1];
    p[1] = d[2] * e2[0] - d[0] * e2[2];
    p[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0.0) return 0;                 /* ray parallel to the plane */
    double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) / det;
    if (!(u >= 0.0 && u <= 1.0)) return 0;
    q[0] = s[1] * e1[2] - s[2] * e1[1];
    q[1] = s[2] * e1[0] - s[0] * e1[2];
    q[2] = s[0] * e1[1] - s[1] * e1[0];
    double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) / det;
    if (!(v >= 0.0 && u + v <= 1.0)) return 0;
    double t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) / det;
    return t > 0.0 && t <= tmax;
}

void orc_dynamic_ao(const float *tris, int64_t n_tris, const float *pos, const float *nrm,
                    const uint64_t *point_id, int64_t count, int rays, double radius, double eps,
                    uint64_t seed, double *out_vis)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < count; ++i) {
        uint64_t pid = point_id ? point_id[i] : (uint64_t)i;
        double n[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        double ln = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int a = 0; a < 3; ++a) n[a] /= ln;
        double o[3];
        for (int a = 0; a < 3; ++a) o[a] = (double)pos[3 * i + a] + eps * n[a];
        int hits = 0;
        for (int k = 0; k < rays; ++k) {
            double d[3];
            orc_cosine_dir(n, orc_uniform(seed, pid, (uint64_t)k, 2, 0),
                           orc_uniform(seed, pid, (uint64_t)k, 2, 1), d);
            for (int64_t j = 0; j < n_tris; ++j)
                if (orc_tri_hit(o, d, tris + 9 * j, radius)) { ++hits; break; }
        }
        out_vis[i] = 1.0 - (double)hits / (double)rays;
    }
}
