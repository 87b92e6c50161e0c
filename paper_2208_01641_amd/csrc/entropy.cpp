// Entropy model and byte-wise rANS coder (host).
//
// The CPU half of the codec (Section III.A-B): integer frequency tables of
// the factorized prior (per channel) and of the Gaussian conditional (per
// scale-table entry), and the entropy coder that turns symbols into the
// per-frame strings.  Byte-wise rANS with a 32-bit state follows the
// published construction (Duda 2013; Giesen 2014): the state lives in
// [2^23, 2^31); before coding a symbol of frequency f the encoder emits
// low bytes while the state is at least 2^15 f, then maps x to
// floor(x / f) 2^16 + x mod f + start.  Streams carry their final state in
// front so that the decoder reads forward.
#include "entropy.h"

#include <math.h>
#include <string.h>

#include <algorithm>

namespace lic {

// --------------------------------------------------------------- density
static inline double softplus(double v) { return log1p(exp(v)); }

double density_logit(const double* prm, double x)
{
    // layer widths 1 -> 3 -> 3 -> 3 -> 1; per layer: matrix (out x in, raw),
    // bias (out), and for the three hidden layers a factor vector (out)
    const int width[5] = {1, 3, 3, 3, 1};
    double cur[3] = {x, 0.0, 0.0};
    int off = 0;
    for (int layer = 0; layer < 4; ++layer) {
        const int nin = width[layer], nout = width[layer + 1];
        const double* mat = prm + off;
        const double* bias = mat + nin * nout;
        const double* fac = bias + nout;
        off += nin * nout + nout + (layer < 3 ? nout : 0);
        double nxt[3];
        for (int o = 0; o < nout; ++o) {
            double u = bias[o];
            for (int i = 0; i < nin; ++i) u += softplus(mat[o * nin + i]) * cur[i];
            if (layer < 3) u = u + tanh(fac[o]) * tanh(u);
            nxt[o] = u;
        }
        for (int o = 0; o < nout; ++o) cur[o] = nxt[o];
    }
    return cur[0];
}

static inline double density_cdf(const double* prm, double x)
{
    return 1.0 / (1.0 + exp(-density_logit(prm, x)));
}

double density_median(const double* prm)
{
    double a = -64.0, b = 64.0;
    for (int step = 0; step < 60; ++step) {
        const double m = 0.5 * (a + b);
        if (density_logit(prm, m) < 0.0) a = m; else b = m;
    }
    return 0.5 * (a + b);
}

void pmf_factorized(const double* prm, double mu, double* p)
{
    for (int s = 0; s < kNumSym; ++s) {
        const int v = s + kSymMin;
        const double upper = (v == 64) ? 1.0 : density_cdf(prm, v + 0.5 + mu);
        const double lower = (v == -64) ? 0.0 : density_cdf(prm, v - 0.5 + mu);
        p[s] = upper - lower;
    }
}

static inline double phi(double u) { return 0.5 * erfc(-u / sqrt(2.0)); }

void pmf_gaussian(double t, double* p)
{
    for (int s = 0; s < kNumSym; ++s) {
        const int v = s + kSymMin;
        p[s] = (v == -64 || v == 64) ? phi(-63.5 / t) : phi((v + 0.5) / t) - phi((v - 0.5) / t);
    }
}

void quantize_pmf(const double* p, uint32_t* f)
{
    const double total = (double)(1u << kPrecBits);
    uint32_t used = 0;
    int mode = 0;
    for (int s = 0; s < kNumSym; ++s) {
        f[s] = 1u + (uint32_t)floor(p[s] * (total - kNumSym));
        used += f[s];
        if (p[s] > p[mode]) mode = s;
    }
    f[mode] += (1u << kPrecBits) - used;
}

void scale_table(double* t)
{
    const double a = log(0.11), b = log(256.0);
    for (int k = 0; k < kScales; ++k) t[k] = exp(a + k * (b - a) / 63.0);
    t[0] = 0.11;
    t[kScales - 1] = 256.0;
}

// ----------------------------------------------------------------- tables
void TableSet::init(int n, const uint32_t* f, bool with_lut)
{
    ntab = n;
    freq.assign(f, f + (size_t)n * kNumSym);
    start.assign((size_t)n * (kNumSym + 1), 0);
    for (int t = 0; t < n; ++t) {
        uint32_t s = 0;
        for (int a = 0; a < kNumSym; ++a) {
            start[(size_t)t * (kNumSym + 1) + a] = s;
            s += freq[(size_t)t * kNumSym + a];
        }
        start[(size_t)t * (kNumSym + 1) + kNumSym] = s;
    }
    // Division by an invariant integer through its reciprocal: with
    // r = ceil(2^64 / f), x r / 2^64 exceeds x / f by less than x / 2^64 <
    // 2^-32, while the fraction of x / f is at most 1 - 1/f <= 1 - 2^-16, so
    // the high word of x r is exactly floor(x / f) for every x < 2^32.
    rcp.assign((size_t)n * kNumSym, 0);
    for (size_t i = 0; i < rcp.size(); ++i) {
        const uint64_t fi = freq[i];
        if (fi > 1) rcp[i] = (~0ull) / fi + 1;     // ceil(2^64 / f) for f >= 2
    }
    bucket.clear();
    if (with_lut) {
        bucket.resize((size_t)n * kBuckets);
        for (int t = 0; t < n; ++t) {
            const uint32_t* st = start.data() + (size_t)t * (kNumSym + 1);
            int a = 0;
            for (int b = 0; b < kBuckets; ++b) {
                const uint32_t slot = (uint32_t)b << kBucketShift;
                while (st[a + 1] <= slot) ++a;
                bucket[(size_t)t * kBuckets + b] = (uint8_t)a;
            }
        }
    }
}

// ------------------------------------------------------------------- rANS
namespace {

struct Writer {
    uint8_t* base;
    long pos;     // bytes are written at decreasing positions
    bool ok = true;
};

inline void enc_put(uint32_t& x, uint32_t f, uint32_t st, uint64_t rcp, Writer& w)
{
    const uint32_t limit = ((kRansLow >> kPrecBits) << 8) * f;   // 2^15 f
    while (x >= limit) {
        if (w.pos == 0) { w.ok = false; return; }
        w.base[--w.pos] = (uint8_t)x;
        x >>= 8;
    }
    // (x / f) 2^16 + x mod f + st = x + st + (x / f)(2^16 - f)
    const uint32_t q = f == 1 ? x : (uint32_t)(((unsigned __int128)x * rcp) >> 64);
    x = x + st + q * ((1u << kPrecBits) - f);
}

inline long enc_finish(uint32_t x, Writer& w, size_t cap)
{
    if (!w.ok || w.pos < 4) return -1;
    w.pos -= 4;
    w.base[w.pos + 0] = (uint8_t)x;
    w.base[w.pos + 1] = (uint8_t)(x >> 8);
    w.base[w.pos + 2] = (uint8_t)(x >> 16);
    w.base[w.pos + 3] = (uint8_t)(x >> 24);
    const long len = (long)cap - w.pos;
    memmove(w.base, w.base + w.pos, (size_t)len);
    return len;
}

inline int find_symbol(const TableSet& T, int t, uint32_t slot)
{
    const uint32_t* st = T.start.data() + (size_t)t * (kNumSym + 1);
    if (!T.bucket.empty()) {
        int a = T.bucket[(size_t)t * kBuckets + (slot >> kBucketShift)];
        while (st[a + 1] <= slot) ++a;
        return a;
    }
    // largest a with st[a] <= slot
    int lo = 0, hi = kNumSym - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st[mid] <= slot) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class TabOf>
long encode_impl(const int8_t* sym, long n, const TableSet& T, uint8_t* out, size_t cap, TabOf tab_of)
{
    Writer w{out, (long)cap};
    uint32_t x = kRansLow;
    for (long i = n - 1; i >= 0; --i) {
        const int t = tab_of(i);
        const int a = (int)sym[i] - kSymMin;
        const size_t k = (size_t)t * kNumSym + a;
        enc_put(x, T.freq[k], T.start[(size_t)t * (kNumSym + 1) + a], T.rcp[k], w);
        if (!w.ok) return -1;
    }
    return enc_finish(x, w, cap);
}

template <class TabOf>
int decode_impl(const uint8_t* in, size_t len, long n, const TableSet& T, int8_t* sym, TabOf tab_of)
{
    if (len < 4) return -1;
    uint32_t x = (uint32_t)in[0] | ((uint32_t)in[1] << 8) | ((uint32_t)in[2] << 16) | ((uint32_t)in[3] << 24);
    size_t pos = 4;
    const uint32_t mask = (1u << kPrecBits) - 1;
    for (long i = 0; i < n; ++i) {
        const int t = tab_of(i);
        const uint32_t slot = x & mask;
        const int a = find_symbol(T, t, slot);
        sym[i] = (int8_t)(a + kSymMin);
        x = T.freq[(size_t)t * kNumSym + a] * (x >> kPrecBits) + slot - T.start[(size_t)t * (kNumSym + 1) + a];
        while (x < kRansLow) {
            if (pos >= len) return -1;
            x = (x << 8) | in[pos++];
        }
    }
    return (x == kRansLow && pos == len) ? 0 : -1;
}

// ------------------------------------------------- interleaved rANS
// K states share one stream of 16-bit words (state range [2^16, 2^32)):
// symbol i is coded by state i mod K, so K independent dependency chains run
// side by side in one thread.  The encoder walks the symbols backwards and
// writes words at decreasing addresses, which leaves them in the reverse of
// the order it pushed them; the decoder, walking forwards, reads each state's
// words in the reverse of that state's pushes from the one shared stream.
// Stream: the K final states (u32 LE, state 0 first), then the words (u16 LE).
// Each state pushes at most one word per symbol (x < 2^32 <= f 2^32 / f), so
// a whole group of K symbols never needs more than 2K bytes: the loops check
// the room once per group and run branch-free inside it.
constexpr uint32_t kWordLow = 1u << 16;

template <int K, class TabOf>
long encode_ileave(const int8_t* sym, long n, const TableSet& T, uint8_t* out, size_t cap, TabOf tab_of)
{
    uint32_t x[K];
    for (int j = 0; j < K; ++j) x[j] = kWordLow;
    long pos = (long)cap;
    const uint32_t* __restrict__ freq = T.freq.data();
    const uint32_t* __restrict__ start = T.start.data();
    const uint64_t* __restrict__ rcp = T.rcp.data();
    // codes symbol i with state xj; with `room` the word is stored unchecked
    auto put = [&](uint32_t& xj, long i, bool room) __attribute__((always_inline)) -> bool {
        const int t = tab_of(i);
        const int a = (int)sym[i] - kSymMin;
        const size_t k = (size_t)t * kNumSym + a;
        const uint32_t f = freq[k];
        const uint32_t push = xj >= (f << kPrecBits) ? 1u : 0u;
        if (!room) {
            if (push) {
                if (pos < 2) return false;
                out[pos - 2] = (uint8_t)xj;
                out[pos - 1] = (uint8_t)(xj >> 8);
            }
        } else {
            out[pos - 2] = (uint8_t)xj;
            out[pos - 1] = (uint8_t)(xj >> 8);
        }
        pos -= 2 * (long)push;
        xj = push ? xj >> 16 : xj;
        const uint32_t q = f == 1 ? xj : (uint32_t)(((unsigned __int128)xj * rcp[k]) >> 64);
        xj = xj + start[(size_t)t * (kNumSym + 1) + a] + q * ((1u << kPrecBits) - f);
        return true;
    };
    const long groups = n / K;
    for (long i = n - 1; i >= groups * K; --i)
        if (!put(x[i % K], i, false)) return -1;
    for (long g = groups - 1; g >= 0; --g) {
        const long i0 = g * K;
        if (pos >= 2L * K) {
#pragma GCC unroll 32
            for (int j = K - 1; j >= 0; --j) put(x[j], i0 + j, true);
        } else {
            for (int j = K - 1; j >= 0; --j)
                if (!put(x[j], i0 + j, false)) return -1;
        }
    }
    if (pos < 4L * K) return -1;
    pos -= 4L * K;
    for (int j = 0; j < K; ++j) {
        out[pos + 4 * j + 0] = (uint8_t)x[j];
        out[pos + 4 * j + 1] = (uint8_t)(x[j] >> 8);
        out[pos + 4 * j + 2] = (uint8_t)(x[j] >> 16);
        out[pos + 4 * j + 3] = (uint8_t)(x[j] >> 24);
    }
    const long len = (long)cap - pos;
    memmove(out, out + pos, (size_t)len);
    return len;
}

template <int K, class TabOf>
int decode_ileave(const uint8_t* in, size_t len, long n, const TableSet& T, int8_t* sym, TabOf tab_of)
{
    if (len < 4u * K) return -1;
    uint32_t x[K];
    for (int j = 0; j < K; ++j)
        x[j] = (uint32_t)in[4 * j] | ((uint32_t)in[4 * j + 1] << 8) | ((uint32_t)in[4 * j + 2] << 16) |
               ((uint32_t)in[4 * j + 3] << 24);
    size_t pos = 4u * K;
    const uint32_t mask = (1u << kPrecBits) - 1;
    const uint32_t* __restrict__ freq = T.freq.data();
    const uint32_t* __restrict__ start = T.start.data();
    // decodes symbol i from state xj; with `room` the word is read unchecked
    auto get = [&](uint32_t& xj, long i, bool room) __attribute__((always_inline)) -> bool {
        const int t = tab_of(i);
        const uint32_t slot = xj & mask;
        const int a = find_symbol(T, t, slot);
        sym[i] = (int8_t)(a + kSymMin);
        xj = freq[(size_t)t * kNumSym + a] * (xj >> kPrecBits) + slot - start[(size_t)t * (kNumSym + 1) + a];
        const bool refill = xj < kWordLow;
        if (!room) {
            if (!refill) return true;
            if (pos + 2 > len) return false;
        }
        const uint32_t w = (uint32_t)in[pos] | ((uint32_t)in[pos + 1] << 8);
        xj = refill ? (xj << 16) | w : xj;
        pos += refill ? 2 : 0;
        return true;
    };
    const long groups = n / K;
    for (long g = 0; g < groups; ++g) {
        const long i0 = g * K;
        if (pos + 2u * K <= len) {
#pragma GCC unroll 32
            for (int j = 0; j < K; ++j) get(x[j], i0 + j, true);
        } else {
            for (int j = 0; j < K; ++j)
                if (!get(x[j], i0 + j, false)) return -1;
        }
    }
    for (long i = groups * K; i < n; ++i)
        if (!get(x[i % K], i, false)) return -1;
    for (int j = 0; j < K; ++j)
        if (x[j] != kWordLow) return -1;
    return pos == len ? 0 : -1;
}

template <class TabOf>
long encode_ileave_k(int K, const int8_t* sym, long n, const TableSet& T, uint8_t* out, size_t cap, TabOf tab_of)
{
    switch (K) {
    case 2: return encode_ileave<2>(sym, n, T, out, cap, tab_of);
    case 4: return encode_ileave<4>(sym, n, T, out, cap, tab_of);
    case 8: return encode_ileave<8>(sym, n, T, out, cap, tab_of);
    case 16: return encode_ileave<16>(sym, n, T, out, cap, tab_of);
    case 32: return encode_ileave<32>(sym, n, T, out, cap, tab_of);
    }
    return -2;
}

template <class TabOf>
int decode_ileave_k(int K, const uint8_t* in, size_t len, long n, const TableSet& T, int8_t* sym, TabOf tab_of)
{
    switch (K) {
    case 2: return decode_ileave<2>(in, len, n, T, sym, tab_of);
    case 4: return decode_ileave<4>(in, len, n, T, sym, tab_of);
    case 8: return decode_ileave<8>(in, len, n, T, sym, tab_of);
    case 16: return decode_ileave<16>(in, len, n, T, sym, tab_of);
    case 32: return decode_ileave<32>(in, len, n, T, sym, tab_of);
    }
    return -2;
}

}  // namespace

bool rans_lanes_valid(int K) { return K == 2 || K == 4 || K == 8 || K == 16 || K == 32; }

long rans_ileave_encode(int K, const int8_t* sym, const uint8_t* tab, long n, const TableSet& T, uint8_t* out,
                        size_t cap)
{
    return encode_ileave_k(K, sym, n, T, out, cap, [tab](long i) { return (int)tab[i]; });
}

long rans_ileave_encode_channel(int K, const int8_t* sym, long n, int C, const TableSet& T, uint8_t* out, size_t cap)
{
    return encode_ileave_k(K, sym, n, T, out, cap, [C](long i) { return (int)(i % C); });
}

int rans_ileave_decode(int K, const uint8_t* in, size_t len, const uint8_t* tab, long n, const TableSet& T,
                       int8_t* sym)
{
    return decode_ileave_k(K, in, len, n, T, sym, [tab](long i) { return (int)tab[i]; });
}

int rans_ileave_decode_channel(int K, const uint8_t* in, size_t len, long n, int C, const TableSet& T, int8_t* sym)
{
    return decode_ileave_k(K, in, len, n, T, sym, [C](long i) { return (int)(i % C); });
}

long rans_encode(const int8_t* sym, const uint8_t* tab, long n, const TableSet& T, uint8_t* out, size_t cap)
{
    return encode_impl(sym, n, T, out, cap, [tab](long i) { return (int)tab[i]; });
}

long rans_encode_channel(const int8_t* sym, long n, int C, const TableSet& T, uint8_t* out, size_t cap)
{
    return encode_impl(sym, n, T, out, cap, [C](long i) { return (int)(i % C); });
}

int rans_decode(const uint8_t* in, size_t len, const uint8_t* tab, long n, const TableSet& T, int8_t* sym)
{
    return decode_impl(in, len, n, T, sym, [tab](long i) { return (int)tab[i]; });
}

int rans_decode_channel(const uint8_t* in, size_t len, long n, int C, const TableSet& T, int8_t* sym)
{
    return decode_impl(in, len, n, T, sym, [C](long i) { return (int)(i % C); });
}

uint32_t fnv1a(const void* data, size_t len)
{
    const uint8_t* p = static_cast<const uint8_t*>(data);
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < len; ++i) {
        h ^= p[i];
        h *= 16777619u;
    }
    return h;
}

// -------------------------------------------------------------- container
static inline void put16(uint8_t* p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static inline void put32(uint8_t* p, uint32_t v)
{
    p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
static inline uint32_t get16(const uint8_t* p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static inline uint32_t get32(const uint8_t* p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

void write_header(uint8_t* out, const StreamHeader& h, uint32_t len_z, const uint32_t* len_y)
{
    memcpy(out, "LICS", 4);
    out[4] = 1;
    out[5] = (uint8_t)h.kind;
    int lg = 0;
    while (h.lanes > 1 && (1 << lg) < h.lanes) ++lg;
    out[6] = (uint8_t)((h.hs_exp & 1) | ((h.norm & 1) << 1) | ((lg & 7) << 2));
    out[7] = (uint8_t)h.S;
    put16(out + 8, h.H);
    put16(out + 10, h.W);
    put16(out + 12, h.N);
    put16(out + 14, h.M);
    put32(out + 16, h.model_id);
    uint8_t* p = out + kHeaderBytes;
    if (h.kind >= 1) { put32(p, len_z); p += 4; }
    for (int s = 0; s < y_streams(h.kind, h.S); ++s, p += 4) put32(p, len_y[s]);
}

bool parse_stream(const uint8_t* bits, size_t len, StreamHeader* h, const uint8_t** z, size_t* len_z,
                  std::vector<const uint8_t*>* y, std::vector<size_t>* len_y, std::string* err)
{
    if (len < kHeaderBytes || memcmp(bits, "LICS", 4) != 0) { *err = "not a LICS bitstream"; return false; }
    if (bits[4] != 1) { *err = "unsupported bitstream version"; return false; }
    h->kind = bits[5];
    h->hs_exp = bits[6] & 1;
    h->norm = (bits[6] >> 1) & 1;
    h->lanes = (bits[6] >> 2) & 7 ? 1 << ((bits[6] >> 2) & 7) : 0;
    if ((bits[6] & 0xe0) != 0 || (h->lanes && !rans_lanes_valid(h->lanes))) { *err = "unknown bitstream flags"; return false; }
    h->S = bits[7];
    h->H = (int)get16(bits + 8);
    h->W = (int)get16(bits + 10);
    h->N = (int)get16(bits + 12);
    h->M = (int)get16(bits + 14);
    h->model_id = get32(bits + 16);
    if (h->kind < 0 || h->kind > 2 || h->S < 1 || h->H < 1 || h->W < 1) { *err = "bad header"; return false; }
    const size_t hs = header_size(h->kind, h->S);
    if (len < hs) { *err = "truncated header"; return false; }
    const uint8_t* p = bits + kHeaderBytes;
    size_t pos = hs;
    *z = nullptr;
    *len_z = 0;
    if (h->kind >= 1) { *len_z = get32(p); p += 4; }
    const int ny = y_streams(h->kind, h->S);
    len_y->resize(ny);
    y->resize(ny);
    size_t total = *len_z;
    for (int s = 0; s < ny; ++s, p += 4) { (*len_y)[s] = get32(p); total += (*len_y)[s]; }
    if (total != len - hs) { *err = "payload length mismatch"; return false; }
    if (h->kind >= 1) { *z = bits + pos; pos += *len_z; }
    for (int s = 0; s < ny; ++s) { (*y)[s] = bits + pos; pos += (*len_y)[s]; }
    return true;
}

}  // namespace lic
