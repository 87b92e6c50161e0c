#include "packing.h"

#include <algorithm>

namespace lic {

namespace {

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

}  // namespace

PackMap pack_map(PackKind kind, int ci, int co, int k, int s, int p, bool w_deconv, int kimg)
{
    PackMap m;
    auto src = [&](int o, int c, int u, int v) -> int32_t {
        return w_deconv ? (int32_t)((((long)c * co + o) * k + u) * k + v)
                        : (int32_t)((((long)o * ci + c) * k + u) * k + v);
    };
    auto add_phase = [&](const PhaseDesc& d, size_t n) {
        m.ph.push_back(d);
        m.off.push_back(m.idx.size());
        m.idx.resize(m.idx.size() + n, -1);
        return m.off.back();
    };

    if (kind == PK_IMG) {
        // one tap whose K runs over the k*k window of the 3 channels
        m.cin = kimg;
        m.cop = 16 * ((co + 15) / 16);
        PhaseDesc d{};
        d.ntaps = 1;
        const size_t base = add_phase(d, (size_t)m.cop * kimg);
        for (int o = 0; o < co; ++o)
            for (int u = 0; u < k; ++u)
                for (int v = 0; v < k; ++v)
                    for (int c = 0; c < ci; ++c) m.idx[base + (size_t)o * kimg + (u * k + v) * ci + c] = src(o, c, u, v);
    } else if (kind == PK_CONV) {
        m.cin = ci;
        m.cop = 16 * ((co + 15) / 16);
        PhaseDesc d{};
        d.ntaps = k * k;
        for (int u = 0; u < k; ++u)
            for (int v = 0; v < k; ++v) {
                d.dy[u * k + v] = (int8_t)(u - p);
                d.dx[u * k + v] = (int8_t)(v - p);
            }
        const size_t base = add_phase(d, (size_t)k * k * m.cop * ci);
        for (int u = 0; u < k; ++u)
            for (int v = 0; v < k; ++v)
                for (int o = 0; o < co; ++o)
                    for (int c = 0; c < ci; ++c)
                        m.idx[base + ((size_t)(u * k + v) * m.cop + o) * ci + c] = src(o, c, u, v);
    } else if (kind == PK_DECONV) {
        // output (s a + py, s b + px) gathers the taps u with (py + p - u)
        // divisible by s, from input row a + (py + p - u) / s
        m.cin = ci;
        m.cop = 16 * ((co + 15) / 16);
        for (int py = 0; py < s; ++py)
            for (int px = 0; px < s; ++px) {
                PhaseDesc d{};
                d.oy = py;
                d.ox = px;
                std::vector<int> us, vs;
                for (int u = 0; u < k; ++u) if ((py + p - u) % s == 0) us.push_back(u);
                for (int v = 0; v < k; ++v) if ((px + p - v) % s == 0) vs.push_back(v);
                d.ntaps = (int)(us.size() * vs.size());
                int t = 0;
                for (int u : us)
                    for (int v : vs) {
                        d.dy[t] = (int8_t)((py + p - u) / s);
                        d.dx[t] = (int8_t)((px + p - v) / s);
                        ++t;
                    }
                const size_t base = add_phase(d, (size_t)d.ntaps * m.cop * ci);
                t = 0;
                for (int u : us)
                    for (int v : vs) {
                        for (int o = 0; o < co; ++o)
                            for (int c = 0; c < ci; ++c)
                                m.idx[base + ((size_t)t * m.cop + o) * ci + c] = src(o, c, u, v);
                        ++t;
                    }
            }
    } else {
        // rows r = 3 (s py + px) + o; tap (dy, dx) of the shared neighbourhood
        // feeds phase py through u = py + p - s dy when 0 <= u < k
        m.cin = ci;
        const int nrow = co * s * s;
        m.cop = 16 * ((nrow + 15) / 16);
        int dmin = 1 << 30, dmax = -(1 << 30);
        for (int py = 0; py < s; ++py) {
            dmin = std::min(dmin, -floor_div(k - 1 - py - p, s));
            dmax = std::max(dmax, floor_div(py + p, s));
        }
        const int nd = dmax - dmin + 1;
        PhaseDesc d{};
        d.ntaps = nd * nd;
        for (int dy = dmin; dy <= dmax; ++dy)
            for (int dx = dmin; dx <= dmax; ++dx) {
                const int t = (dy - dmin) * nd + (dx - dmin);
                d.dy[t] = (int8_t)dy;
                d.dx[t] = (int8_t)dx;
            }
        const size_t base = add_phase(d, (size_t)d.ntaps * m.cop * ci);
        for (int dy = dmin; dy <= dmax; ++dy)
            for (int dx = dmin; dx <= dmax; ++dx) {
                const int t = (dy - dmin) * nd + (dx - dmin);
                for (int py = 0; py < s; ++py)
                    for (int px = 0; px < s; ++px) {
                        const int u = py + p - s * dy, v = px + p - s * dx;
                        if (u < 0 || u >= k || v < 0 || v >= k) continue;
                        for (int o = 0; o < co; ++o) {
                            const int r = co * (s * py + px) + o;
                            for (int c = 0; c < ci; ++c) m.idx[base + ((size_t)t * m.cop + r) * ci + c] = src(o, c, u, v);
                        }
                    }
            }
    }
    m.bias_idx.assign(m.cop, -1);
    const int nrow = kind == PK_ROWS ? co * s * s : co;
    for (int r = 0; r < nrow; ++r) m.bias_idx[r] = r % co;
    return m;
}

PackMap pack_map_checkerboard(int ci, int co, int k, int part, bool pair_rows)
{
    PackMap m;
    m.cin = ci;
    m.cop = 16 * ((co + 15) / 16);
    const int p = k / 2;
    auto row_of = [&](int o) { return pair_rows ? (o < co / 2 ? 2 * o : 2 * (o - co / 2) + 1) : o; };
    const int phases[2][2][2] = {{{0, 0}, {1, 1}}, {{0, 1}, {1, 0}}};
    for (int f = 0; f < 2; ++f) {
        PhaseDesc d{};
        d.oy = phases[part][f][0];
        d.ox = phases[part][f][1];
        std::vector<int> us, vs;
        for (int u = 0; u < k; ++u)
            for (int v = 0; v < k; ++v)
                if (k == 1 || (u + v - 2 * p) % 2 != 0) {
                    us.push_back(u);
                    vs.push_back(v);
                }
        d.ntaps = (int)us.size();
        for (int t = 0; t < d.ntaps; ++t) {
            d.dy[t] = (int8_t)(d.oy + us[t] - p);
            d.dx[t] = (int8_t)(d.ox + vs[t] - p);
        }
        m.ph.push_back(d);
        m.off.push_back(m.idx.size());
        const size_t base = m.idx.size();
        m.idx.resize(base + (size_t)d.ntaps * m.cop * ci, -1);
        for (int t = 0; t < d.ntaps; ++t)
            for (int o = 0; o < co; ++o)
                for (int c = 0; c < ci; ++c)
                    m.idx[base + ((size_t)t * m.cop + row_of(o)) * ci + c] =
                        (int32_t)((((long)o * ci + c) * k + us[t]) * k + vs[t]);
    }
    m.bias_idx.assign(m.cop, -1);
    for (int o = 0; o < co; ++o) m.bias_idx[row_of(o)] = o;
    return m;
}

}  // namespace lic
