/*
 * FP64 reference ("oracle") for the learned-image-codec hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library: it is written from the definitions of the operations,
 * as plain loops in double precision, with no blocking or reordering beyond
 * what each definition states.
 *
 * Operations and where they come from
 *   - convolution and transposed convolution: the analysis / synthesis
 *     transforms g_a, g_s and the hyper transforms h_a, h_s of the
 *     factorized-prior and scale-hyperprior codecs (Section III.A-B, Fig. 1).
 *   - GDN / IGDN, the normalisation the paper names as the main overhead of
 *     those transforms (Section IV.C): y_i = x_i / sqrt(beta_i + sum_j
 *     gamma_ij x_j^2), and x_i * sqrt(...) for the inverse; and 1DN, the
 *     cheaper normalisation of implementation C (same section), read as
 *     y_i = x_i / (beta_i + sum_j gamma_ij |x_j|) and x_i * (...).
 *   - the per-channel factorized density (entropy bottleneck of the
 *     factorized prior, Section III.A), its median, and the integer
 *     frequency tables with 16-bit precision.
 *   - Gaussian tables over a 64-entry log-spaced scale table (the scale
 *     hyperprior's conditional model, Section III.B).
 *   - a byte-wise 32-bit rANS coder: the CPU entropy (de)coding workload of
 *     Section III.A-B.  The paper uses a third-party coder; this is the
 *     published byte-wise rANS construction (Duda 2013, Giesen 2014).
 *
 * Parity status: every function here is pinned by the CPU tests (brute
 * force, closed forms, identities, round trips); see the test files.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* OpenMP threads of the parallel loops below (timing runs on a chosen core
 * count); returns the count in effect. */
int or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Convolution (NCHW, zero outside the input)                                */
/*   out[o,i,j] = b_o + sum_{c,u,v} w[o,c,u,v] * in[c, s*i+u-p, s*j+v-p]    */
/* ------------------------------------------------------------------------ */
double or_conv2d_at(const double* in, int C, int H, int W,
                    const double* w, const double* b, int k, int s, int p,
                    int o, int i, int j)
{
    double acc = b ? b[o] : 0.0;
    for (int c = 0; c < C; ++c)
        for (int u = 0; u < k; ++u) {
            int r = s * i + u - p;
            if (r < 0 || r >= H) continue;
            for (int v = 0; v < k; ++v) {
                int q = s * j + v - p;
                if (q < 0 || q >= W) continue;
                acc += w[(((long)o * C + c) * k + u) * k + v] * in[((long)c * H + r) * W + q];
            }
        }
    return acc;
}

void or_conv2d(const double* in, int C, int H, int W,
               const double* w, const double* b, int Co, int k, int s, int p,
               double* out, int Ho, int Wo)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int o = 0; o < Co; ++o)
        for (int i = 0; i < Ho; ++i)
            for (int j = 0; j < Wo; ++j)
                out[((long)o * Ho + i) * Wo + j] = or_conv2d_at(in, C, H, W, w, b, k, s, p, o, i, j);
}

/* ------------------------------------------------------------------------ */
/* Transposed convolution (weights [C_in, C_out, k, k])                     */
/*   out[o,i,j] = b_o + sum_c sum_{u,v: (i+p-u) and (j+p-v) divisible by s} */
/*                w[c,o,u,v] * in[c, (i+p-u)/s, (j+p-v)/s]                  */
/*   over valid input indices; H_out = (H-1)s - 2p + k + output_padding.    */
/* ------------------------------------------------------------------------ */
double or_deconv2d_at(const double* in, int C, int H, int W,
                      const double* w, const double* b, int Co, int k, int s, int p,
                      int o, int i, int j)
{
    /* the taps u with (i + p - u) divisible by s are u0, u0 + s, ... with  */
    /* u0 = (i + p) mod s (likewise v); the others contribute nothing      */
    const int u0 = (i + p) % s, v0 = (j + p) % s;
    double acc = b ? b[o] : 0.0;
    for (int c = 0; c < C; ++c)
        for (int u = u0; u < k; u += s) {
            int ti = i + p - u;
            if (ti < 0) continue;
            int r = ti / s;
            if (r >= H) continue;
            for (int v = v0; v < k; v += s) {
                int tj = j + p - v;
                if (tj < 0) continue;
                int q = tj / s;
                if (q >= W) continue;
                acc += w[(((long)c * Co + o) * k + u) * k + v] * in[((long)c * H + r) * W + q];
            }
        }
    return acc;
}

void or_deconv2d(const double* in, int C, int H, int W,
                 const double* w, const double* b, int Co, int k, int s, int p,
                 double* out, int Ho, int Wo)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int o = 0; o < Co; ++o)
        for (int i = 0; i < Ho; ++i)
            for (int j = 0; j < Wo; ++j)
                out[((long)o * Ho + i) * Wo + j] = or_deconv2d_at(in, C, H, W, w, b, Co, k, s, p, o, i, j);
}

/* All output channels at a list of output positions (i, j): out[n][Co]. */
void or_conv2d_points(const double* in, int C, int H, int W,
                      const double* w, const double* b, int Co, int k, int s, int p,
                      int npts, const int* ij, double* out)
{
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < npts; ++q)
        for (int o = 0; o < Co; ++o)
            out[(long)q * Co + o] = or_conv2d_at(in, C, H, W, w, b, k, s, p, o, ij[2 * q], ij[2 * q + 1]);
}

void or_deconv2d_points(const double* in, int C, int H, int W,
                        const double* w, const double* b, int Co, int k, int s, int p,
                        int npts, const int* ij, double* out)
{
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < npts; ++q)
        for (int o = 0; o < Co; ++o)
            out[(long)q * Co + o] = or_deconv2d_at(in, C, H, W, w, b, Co, k, s, p, o, ij[2 * q], ij[2 * q + 1]);
}

/* Weight gradient of a transposed convolution (weights [C_in, C_out, k, k]) */
/* for one image:  dW[c,o,u,v] += sum_{a,b} x[c,a,b] dy[o, s a + u - p, s b + v - p] */
/* over output positions inside dy; db[o] += sum of dy[o].  Accumulates.    */
void or_deconv2d_wgrad(const double* x, int C, int H, int W, const double* dy, int Co, int Ho, int Wo,
                       int k, int s, int p, double* dw, double* db)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c)
        for (int o = 0; o < Co; ++o)
            for (int u = 0; u < k; ++u)
                for (int v = 0; v < k; ++v) {
                    double acc = 0.0;
                    for (int a = 0; a < H; ++a) {
                        int i = s * a + u - p;
                        if (i < 0 || i >= Ho) continue;
                        for (int b = 0; b < W; ++b) {
                            int j = s * b + v - p;
                            if (j < 0 || j >= Wo) continue;
                            acc += x[((long)c * H + a) * W + b] * dy[((long)o * Ho + i) * Wo + j];
                        }
                    }
                    dw[(((long)c * Co + o) * k + u) * k + v] += acc;
                }
    if (db)
        for (int o = 0; o < Co; ++o) {
            double acc = 0.0;
            for (long q = 0; q < (long)Ho * Wo; ++q) acc += dy[(long)o * Ho * Wo + q];
            db[o] += acc;
        }
}

/* One AdamW step with decoupled weight decay and bias correction, step t  */
/* counted from 1:  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;         */
/* w <- w (1 - lr wd) - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).    */
void or_adamw(double* w, double* m, double* v, const double* g, long n, long t,
              double lr, double b1, double b2, double eps, double wd)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] = w[i] * (1.0 - lr * wd) - lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* GDN / IGDN, per pixel over channels.  x and out are [C][HW] planes.      */
/*   n_i = beta_i + sum_j gamma[i][j] x_j^2                                 */
/*   GDN: x_i / sqrt(n_i)      IGDN: x_i * sqrt(n_i)                        */
/* ------------------------------------------------------------------------ */
void or_gdn(const double* x, int C, long HW, const double* beta, const double* gamma,
            int inverse, double* out)
{
#pragma omp parallel for schedule(static)
    for (long q = 0; q < HW; ++q)
        for (int i = 0; i < C; ++i) {
            double n = beta[i];
            for (int j = 0; j < C; ++j) {
                double xj = x[(long)j * HW + q];
                n += gamma[(long)i * C + j] * xj * xj;
            }
            double xi = x[(long)i * HW + q];
            out[(long)i * HW + q] = inverse ? xi * sqrt(n) : xi / sqrt(n);
        }
}

/* ------------------------------------------------------------------------ */
/* 1DN, the cheaper normalisation that replaces GDN in the paper's          */
/* implementation C (Section IV.C; the paper names it and cites it but      */
/* prints no formula).  Read as GDN with the square of the channel mixing   */
/* replaced by the absolute value and no square root:                       */
/*   n_i = beta_i + sum_j gamma[i][j] |x_j|                                 */
/*   forward: x_i / n_i      inverse: x_i * n_i                             */
/* ------------------------------------------------------------------------ */
void or_gdn1(const double* x, int C, long HW, const double* beta, const double* gamma,
             int inverse, double* out)
{
#pragma omp parallel for schedule(static)
    for (long q = 0; q < HW; ++q)
        for (int i = 0; i < C; ++i) {
            double n = beta[i];
            for (int j = 0; j < C; ++j) n += gamma[(long)i * C + j] * fabs(x[(long)j * HW + q]);
            double xi = x[(long)i * HW + q];
            out[(long)i * HW + q] = inverse ? xi * n : xi / n;
        }
}

/* ------------------------------------------------------------------------ */
/* Factorized density of one channel (the non-parametric cumulative of the  */
/* factorized-prior entropy bottleneck).  Raw parameters, 43 doubles:       */
/*   H1(3x1) b1(3) a1(3) H2(3x3) b2(3) a2(3) H3(3x3) b3(3) a3(3) H4(1x3) b4 */
/* Layer k: u = softplus(Hraw_k) f + b_k; hidden layers apply               */
/*   g(u) = u + tanh(a_k) * tanh(u); the last layer's u is the logit of the */
/*   cumulative, c(x) = sigmoid(logit).                                     */
/* ------------------------------------------------------------------------ */
static double softplus(double x) { return log1p(exp(x)); }

double or_density_logit(const double* prm, double x)
{
    static const int dims[5] = {1, 3, 3, 3, 1};
    double f[3] = {x, 0.0, 0.0}, g[3];
    const double* q = prm;
    for (int k = 0; k < 4; ++k) {
        int din = dims[k], dout = dims[k + 1];
        const double* Hraw = q;  q += din * dout;
        const double* bias = q;  q += dout;
        const double* fac = 0;
        if (k < 3) { fac = q; q += dout; }
        for (int r = 0; r < dout; ++r) {
            double u = bias[r];
            for (int c = 0; c < din; ++c) u += softplus(Hraw[r * din + c]) * f[c];
            if (k < 3) u = u + tanh(fac[r]) * tanh(u);
            g[r] = u;
        }
        for (int r = 0; r < dout; ++r) f[r] = g[r];
    }
    return f[0];
}

double or_density_cdf(const double* prm, double x)
{
    return 1.0 / (1.0 + exp(-or_density_logit(prm, x)));
}

/* Median: bisection on [-64, 64], 60 halvings, c(mid) < 1/2 <=> logit < 0. */
double or_density_median(const double* prm)
{
    double lo = -64.0, hi = 64.0;
    for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi);
        if (or_density_logit(prm, mid) < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Probability mass over the 129 symbols j = -64..64 (index j + 64).        */
/* ------------------------------------------------------------------------ */
#define OR_NSYM 129
#define OR_SYM_MIN (-64)
#define OR_PREC 16

/* factorized: p_j = c(j + 1/2 + mu) - c(j - 1/2 + mu); the edge bins take  */
/* the tails, p_-64 = c(-63.5 + mu), p_64 = 1 - c(63.5 + mu).               */
void or_pmf_factorized(const double* prm, double mu, double* p)
{
    for (int a = 0; a < OR_NSYM; ++a) {
        int j = a + OR_SYM_MIN;
        double hi = (j == 64) ? 1.0 : or_density_cdf(prm, j + 0.5 + mu);
        double lo = (j == -64) ? 0.0 : or_density_cdf(prm, j - 0.5 + mu);
        p[a] = hi - lo;
    }
}

/* standard normal cumulative from the complementary error function */
static double std_normal_cdf(double u) { return 0.5 * erfc(-u / sqrt(2.0)); }

/* zero-mean Gaussian of scale t: p_j = Phi((j+1/2)/t) - Phi((j-1/2)/t),    */
/* edge bins take the tails: p_-64 = Phi(-63.5/t), p_64 = Phi(-63.5/t).     */
void or_pmf_gaussian(double t, double* p)
{
    for (int a = 0; a < OR_NSYM; ++a) {
        int j = a + OR_SYM_MIN;
        if (j == -64 || j == 64) p[a] = std_normal_cdf(-63.5 / t);
        else p[a] = std_normal_cdf((j + 0.5) / t) - std_normal_cdf((j - 0.5) / t);
    }
}

/* Integer frequencies summing to 2^16: f_j = 1 + floor(p_j (2^16 - 129));   */
/* the remainder goes to the most probable symbol (lowest index on a tie).  */
void or_quantize_pmf(const double* p, uint32_t* f)
{
    const double R = (double)(1u << OR_PREC);
    uint32_t sum = 0;
    int best = 0;
    for (int a = 0; a < OR_NSYM; ++a) {
        f[a] = 1u + (uint32_t)floor(p[a] * (R - OR_NSYM));
        sum += f[a];
        if (p[a] > p[best]) best = a;
    }
    f[best] += (1u << OR_PREC) - sum;
}

/* 64 log-spaced scales from 0.11 to 256, both endpoints exact. */
void or_scale_table(double* t)
{
    const double lo = log(0.11), hi = log(256.0);
    for (int k = 0; k < 64; ++k) t[k] = exp(lo + k * (hi - lo) / 63.0);
    t[0] = 0.11;
    t[63] = 256.0;
}

/* Scale index: s <- max(s, t_0); idx = #{k in [0, 62] : t_k < s}. */
int or_scale_index(const double* t, double s)
{
    if (s < t[0]) s = t[0];
    int idx = 0;
    for (int k = 0; k <= 62; ++k)
        if (t[k] < s) ++idx;
    return idx;
}

/* ------------------------------------------------------------------------ */
/* Byte-wise rANS, 32-bit state, lower bound L = 2^23, 16-bit frequencies.  */
/* Symbols are alphabet indices 0..128; tab[i] selects the table of symbol  */
/* i; freq is [ntab][129].  Encoding runs over the symbols in reverse, the  */
/* bytes are produced back to front, and the final state is written as 4    */
/* little-endian bytes at the front, so decoding reads forward.             */
/* Returns the stream length, or -1 if it does not fit in cap.              */
/* ------------------------------------------------------------------------ */
#define OR_RANS_L (1u << 23)

static uint32_t cum_start(const uint32_t* f, int a)
{
    uint32_t s = 0;
    for (int i = 0; i < a; ++i) s += f[i];
    return s;
}

long or_rans_encode(const int32_t* sym, const int32_t* tab, long n,
                    const uint32_t* freq, uint8_t* out, long cap)
{
    long pos = cap;
    uint32_t x = OR_RANS_L;
    for (long i = n - 1; i >= 0; --i) {
        const uint32_t* f = freq + (long)tab[i] * OR_NSYM;
        uint32_t fs = f[sym[i]];
        uint32_t st = cum_start(f, sym[i]);
        uint32_t x_max = ((OR_RANS_L >> OR_PREC) << 8) * fs;
        while (x >= x_max) {
            if (pos == 0) return -1;
            out[--pos] = (uint8_t)(x & 0xffu);
            x >>= 8;
        }
        x = ((x / fs) << OR_PREC) + (x % fs) + st;
    }
    if (pos < 4) return -1;
    pos -= 4;
    out[pos + 0] = (uint8_t)(x);
    out[pos + 1] = (uint8_t)(x >> 8);
    out[pos + 2] = (uint8_t)(x >> 16);
    out[pos + 3] = (uint8_t)(x >> 24);
    long len = cap - pos;
    memmove(out, out + pos, (size_t)len);
    return len;
}

/* Decodes n symbols; returns 0 on success, -1 if the stream is truncated, */
/* -2 if it does not end in state L with every byte consumed.              */
int or_rans_decode(const uint8_t* in, long len, const int32_t* tab, long n,
                   const uint32_t* freq, int32_t* sym)
{
    if (len < 4) return -1;
    uint32_t x = (uint32_t)in[0] | ((uint32_t)in[1] << 8) | ((uint32_t)in[2] << 16) | ((uint32_t)in[3] << 24);
    long pos = 4;
    for (long i = 0; i < n; ++i) {
        const uint32_t* f = freq + (long)tab[i] * OR_NSYM;
        uint32_t slot = x & ((1u << OR_PREC) - 1);
        int a = 0;
        uint32_t st = 0;
        while (a < OR_NSYM - 1 && st + f[a] <= slot) { st += f[a]; ++a; }
        sym[i] = a;
        x = f[a] * (x >> OR_PREC) + slot - st;
        while (x < OR_RANS_L) {
            if (pos >= len) return -1;
            x = (x << 8) | in[pos++];
        }
    }
    if (x != OR_RANS_L || pos != len) return -2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Interleaved word-wise rANS (the faster entropy coding the paper points   */
/* to in Sections II and VII; the construction is Giesen's interleaved      */
/* rANS, 2014).  K coder states share one stream.  Each state is 32 bits    */
/* with lower bound L = 2^16 and exchanges 16-bit words with the stream;    */
/* frequencies have 16-bit precision, as above.  Symbol i is coded by state */
/* i mod K.  Encoding runs over the symbols in reverse: before symbol i its */
/* state x pushes its low 16 bits and shifts right by 16 if x >= f 2^16,     */
/* then x <- (x / f) 2^16 + x mod f + start.  The stream is the K final     */
/* states (u32 little-endian, state 0 first) followed by the pushed words   */
/* in the reverse of their push order (u16 little-endian).  Decoding runs   */
/* forward: slot = x mod 2^16, the symbol a with start_a <= slot <          */
/* start_a + f_a, x <- f_a (x / 2^16) + slot - start_a, then one word is    */
/* read, x <- x 2^16 + word, if x < 2^16.  Because every state reads its    */
/* words in the reverse of the order the encoder pushed them, the one       */
/* shared stream serves all K states.  At the end every state is L again    */
/* and every word has been read.                                            */
/* Returns the stream length in bytes, or -1 if it does not fit in cap.     */
/* ------------------------------------------------------------------------ */
#define OR_RANS16_L (1u << 16)

long or_rans_ileave_encode(const int32_t* sym, const int32_t* tab, long n, int K,
                           const uint32_t* freq, uint8_t* out, long cap)
{
    uint32_t x[64];
    if (K < 1 || K > 64) return -1;
    for (int j = 0; j < K; ++j) x[j] = OR_RANS16_L;
    long pos = cap;
    for (long i = n - 1; i >= 0; --i) {
        const int j = (int)(i % K);
        const uint32_t* f = freq + (long)tab[i] * OR_NSYM;
        uint32_t fs = f[sym[i]];
        uint32_t st = cum_start(f, sym[i]);
        if (x[j] >= (fs << 16)) {
            if (pos < 2) return -1;
            pos -= 2;
            out[pos + 0] = (uint8_t)(x[j]);
            out[pos + 1] = (uint8_t)(x[j] >> 8);
            x[j] >>= 16;
        }
        x[j] = ((x[j] / fs) << OR_PREC) + (x[j] % fs) + st;
    }
    if (pos < 4L * K) return -1;
    pos -= 4L * K;
    for (int j = 0; j < K; ++j) {
        out[pos + 4 * j + 0] = (uint8_t)(x[j]);
        out[pos + 4 * j + 1] = (uint8_t)(x[j] >> 8);
        out[pos + 4 * j + 2] = (uint8_t)(x[j] >> 16);
        out[pos + 4 * j + 3] = (uint8_t)(x[j] >> 24);
    }
    long len = cap - pos;
    memmove(out, out + pos, (size_t)len);
    return len;
}

/* Returns 0 on success, -1 if the stream is truncated, -2 if it does not   */
/* end with every state at L and every word read.                           */
int or_rans_ileave_decode(const uint8_t* in, long len, const int32_t* tab, long n, int K,
                          const uint32_t* freq, int32_t* sym)
{
    uint32_t x[64];
    if (K < 1 || K > 64 || len < 4L * K) return -1;
    for (int j = 0; j < K; ++j)
        x[j] = (uint32_t)in[4 * j] | ((uint32_t)in[4 * j + 1] << 8) | ((uint32_t)in[4 * j + 2] << 16) |
               ((uint32_t)in[4 * j + 3] << 24);
    long pos = 4L * K;
    for (long i = 0; i < n; ++i) {
        const int j = (int)(i % K);
        const uint32_t* f = freq + (long)tab[i] * OR_NSYM;
        uint32_t slot = x[j] & ((1u << OR_PREC) - 1);
        int a = 0;
        uint32_t st = 0;
        while (a < OR_NSYM - 1 && st + f[a] <= slot) { st += f[a]; ++a; }
        sym[i] = a;
        x[j] = f[a] * (x[j] >> OR_PREC) + slot - st;
        if (x[j] < OR_RANS16_L) {
            if (pos + 2 > len) return -1;
            x[j] = (x[j] << 16) | (uint32_t)in[pos] | ((uint32_t)in[pos + 1] << 8);
            pos += 2;
        }
    }
    for (int j = 0; j < K; ++j)
        if (x[j] != OR_RANS16_L) return -2;
    return pos == len ? 0 : -2;
}
