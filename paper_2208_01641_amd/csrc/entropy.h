// Host-side entropy model and coder: factorized-density and Gaussian
// frequency tables (16-bit), byte-wise rANS, and the bitstream container.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace lic {

constexpr int kNumSym = 129;          // symbols -64..64, stored as value + 64
constexpr int kSymMin = -64;
constexpr int kPrecBits = 16;         // frequencies sum to 2^16
constexpr uint32_t kRansLow = 1u << 23;
constexpr int kBucketShift = 6;        // decoder buckets of 64 slots
constexpr int kBuckets = 1 << (kPrecBits - kBucketShift);
constexpr int kDensityParams = 43;    // raw parameters of one channel's density
constexpr int kScales = 64;

// Logit of the cumulative of one channel's factorized density (1-3-3-3-1
// network with softplus-positive matrices and tanh non-linearities).
double density_logit(const double* prm, double x);
// Channel median by 60-step bisection on [-64, 64].
double density_median(const double* prm);
// Probability of each symbol j = -64..64 under the density, offset by mu.
void pmf_factorized(const double* prm, double mu, double* p);
// Probability of each symbol under a zero-mean Gaussian of scale t.
void pmf_gaussian(double t, double* p);
// 16-bit integer frequencies (every symbol >= 1, remainder to the mode).
void quantize_pmf(const double* p, uint32_t* f);
// 64 log-spaced scales 0.11 .. 256 (endpoints exact).
void scale_table(double* t);

// A set of frequency tables with cumulative starts and, optionally, a
// slot -> symbol lookup for decoding.
struct TableSet {
    int ntab = 0;
    std::vector<uint32_t> freq;    // [ntab][129]
    std::vector<uint32_t> start;   // [ntab][130]
    // encoder: x / f as the high word of x * rcp (rcp = ceil(2^64 / f), 0 for f = 1)
    std::vector<uint64_t> rcp;     // [ntab][129]
    // decoder: symbol holding the first slot of each 64-slot bucket (empty:
    // binary search over start); a short forward scan finishes the search
    std::vector<uint8_t> bucket;   // [ntab][1024]
    void init(int n, const uint32_t* f, bool with_lut);
};

// Symbols are the int8 values -64..64 the GPU epilogues write; the coder
// works on alphabet indices value + 64.
// Returns bytes written, or -1 if cap is too small.
long rans_encode(const int8_t* sym, const uint8_t* tab, long n, const TableSet& T,
                 uint8_t* out, size_t cap);
// Encodes symbols whose table is the channel (c = position % C): z, factorized y.
long rans_encode_channel(const int8_t* sym, long n, int C, const TableSet& T,
                         uint8_t* out, size_t cap);
// Returns 0, or -1 on a truncated / inconsistent stream.
int rans_decode(const uint8_t* in, size_t len, const uint8_t* tab, long n, const TableSet& T,
                int8_t* sym);
int rans_decode_channel(const uint8_t* in, size_t len, long n, int C, const TableSet& T,
                        int8_t* sym);

// Interleaved word-wise rANS with K states (K = 2, 4, 8, 16 or 32; symbol i
// on state i mod K, 32-bit states in [2^16, 2^32), 16-bit words, one shared
// stream: the K final states, then the words).  Same return values as above;
// a stream of n symbols takes at most 2 n + 4 K bytes.
bool rans_lanes_valid(int K);
long rans_ileave_encode(int K, const int8_t* sym, const uint8_t* tab, long n, const TableSet& T, uint8_t* out,
                        size_t cap);
long rans_ileave_encode_channel(int K, const int8_t* sym, long n, int C, const TableSet& T, uint8_t* out, size_t cap);
int rans_ileave_decode(int K, const uint8_t* in, size_t len, const uint8_t* tab, long n, const TableSet& T,
                       int8_t* sym);
int rans_ileave_decode_channel(int K, const uint8_t* in, size_t len, long n, int C, const TableSet& T, int8_t* sym);

uint32_t fnv1a(const void* data, size_t len);

// ---------------------------------------------------------------- container
// flags: bit 0 exp output of h_s, bit 1 1DN instead of GDN, bits 2..4 log2 of
// the interleaved rANS states (0: byte-wise single-state rANS), bits 5..7 zero
struct StreamHeader {
    int kind = 1, hs_exp = 1, S = 1, H = 0, W = 0, N = 0, M = 0;
    int norm = 0, lanes = 0;
    uint32_t model_id = 0;
};
constexpr size_t kHeaderBytes = 20;
// room beyond 2 bytes per symbol that one rANS stream may need (the final
// states: 4 bytes byte-wise, 4 K interleaved)
constexpr size_t kStreamSlack = 160;
// y streams of a bitstream: S row slices, twice for the context model (the
// anchors' S slices, then the other positions' S slices)
inline int y_streams(int kind, int S) { return kind == 2 ? 2 * S : S; }
inline size_t header_size(int kind, int S) { return kHeaderBytes + 4u * (y_streams(kind, S) + (kind >= 1 ? 1 : 0)); }
// len_y: y_streams(h.kind, h.S) lengths
void write_header(uint8_t* out, const StreamHeader& h, uint32_t len_z, const uint32_t* len_y);
// Validates and returns the payload spans; false on any inconsistency.
bool parse_stream(const uint8_t* bits, size_t len, StreamHeader* h,
                  const uint8_t** z, size_t* len_z, std::vector<const uint8_t*>* y,
                  std::vector<size_t>* len_y, std::string* err);

}  // namespace lic
