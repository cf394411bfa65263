// Host-side constants of the Ozaki-II scheme: moduli (Algorithm 1 Step I),
// CRT weights s_l = (P/p_l) q_l (Step II and Step V-v), and the integer
// thresholds that decide the scaling exponents (Section III-B).
//
// A tiny unsigned big-integer type is enough: P < 2^190 for N <= 24.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace ozc {
namespace {

struct Big {
    std::vector<uint32_t> w;  // little-endian 32-bit words, no leading zero words

    explicit Big(uint64_t v = 0) {
        if (v) w.push_back((uint32_t)v);
        if (v >> 32) w.push_back((uint32_t)(v >> 32));
    }
    void trim() {
        while (!w.empty() && w.back() == 0) w.pop_back();
    }
    int bitlen() const {
        if (w.empty()) return 0;
        return 32 * (int)(w.size() - 1) + (32 - __builtin_clz(w.back()));
    }
    int bit(int b) const {
        size_t i = (size_t)b / 32;
        return i < w.size() ? (int)((w[i] >> (b % 32)) & 1u) : 0;
    }
    Big mul(uint32_t s) const {
        Big r;
        uint64_t c = 0;
        for (uint32_t x : w) {
            c += (uint64_t)x * s;
            r.w.push_back((uint32_t)c);
            c >>= 32;
        }
        if (c) r.w.push_back((uint32_t)c);
        r.trim();
        return r;
    }
    uint32_t mod(uint32_t s) const {
        uint64_t r = 0;
        for (size_t i = w.size(); i-- > 0;) r = ((r << 32) | w[i]) % s;
        return (uint32_t)r;
    }
    Big div(uint32_t s) const {
        Big q;
        q.w.resize(w.size());
        uint64_t r = 0;
        for (size_t i = w.size(); i-- > 0;) {
            uint64_t cur = (r << 32) | w[i];
            q.w[i] = (uint32_t)(cur / s);
            r = cur % s;
        }
        q.trim();
        return q;
    }
    Big minus1() const {  // this - 1, this > 0
        Big r = *this;
        for (auto &x : r.w) {
            if (x--) break;
        }
        r.trim();
        return r;
    }
    // floor(this * 2^e) for any integer e
    Big shift(int e) const {
        Big r;
        int bl = bitlen();
        if (bl == 0) return r;
        int nb = bl + e;
        if (nb <= 0) return r;
        r.w.assign((size_t)(nb + 31) / 32, 0u);
        for (int b = std::max(0, -e); b < bl; ++b)
            if (bit(b)) r.w[(size_t)(b + e) / 32] |= 1u << ((b + e) % 32);
        r.trim();
        return r;
    }
    uint64_t clamp_u64() const {
        if (bitlen() > 64) return UINT64_MAX;
        uint64_t v = 0;
        for (size_t i = w.size(); i-- > 0;) v = (v << 32) | w[i];
        return v;
    }
    // bits [lo, lo + n) as an integer (n <= 32)
    uint32_t bits(int lo, int n) const {
        uint32_t v = 0;
        for (int b = 0; b < n; ++b) v |= (uint32_t)bit(lo + b) << b;
        return v;
    }
    double approx() const {  // close to the value (not necessarily correctly rounded)
        double v = 0.0;
        for (size_t i = w.size(); i-- > 0;) v = v * 4294967296.0 + (double)w[i];
        return v;
    }
};

int gcd(int a, int b) {
    while (b) {
        int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

uint32_t inverse_mod(uint32_t a, uint32_t p) {  // a * x = 1 (mod p), p <= 256
    for (uint32_t x = 1; x < p; ++x)
        if ((a * x) % p == 1u) return x;
    return 0;
}

}  // namespace

// Bits [38 c, 38 c + 38) of v as an exact double.
static double chunk(const Big &v, int c) {
    constexpr int h = kChunkBits / 2;
    return (double)v.bits(kChunkBits * c, h) + (double)v.bits(kChunkBits * c + h, h) * (double)(1u << h);
}

void build_tables(NTable *tables) {
    // Step I: greedy descending pairwise-coprime integers <= 256.
    std::vector<int> all;
    for (int c = 256; (int)all.size() < kMaxModuli; --c) {
        bool ok = true;
        for (int p : all) ok = ok && gcd(c, p) == 1;
        if (ok) all.push_back(c);
    }
    for (int n = 1; n <= kMaxModuli; ++n) {
        NTable &t = tables[n - 1];
        memset(&t, 0, sizeof(t));
        t.n = n;
        Big P(1);
        for (int l = 0; l < n; ++l) P = P.mul((uint32_t)all[l]);
        const int pbits = P.bitlen();
        // at most kMaxChunks for N <= 24; a larger count would make every CRT launch
        // fail with an invalid-value error rather than overrun the tables
        t.nchunks = (pbits + kChunkBits - 1) / kChunkBits;
        for (int c = 0; c < std::min(t.nchunks, kMaxChunks); ++c) t.Pchunk[c] = chunk(P, c);
        t.P_approx = P.approx();
        t.inv_P = 1.0 / t.P_approx;

        const Big Pm1 = P.minus1();
        const int lb = Pm1.bitlen() - 1;  // floor(log2(P - 1))
        // fast mode: t <= P'_fast - 1 with P'_fast = log2(P-1)/2 - 1.5  <=>  2^(2t+5) <= P - 1
        t.fast_tmax = (int)std::floor((lb - 5) / 2.0);
        // accurate mode: 2 * X * 4^t <= P - 1 with X >= 1
        t.accu_thi = (int)std::floor((lb - 1) / 2.0);
        for (int d = 0; d < kThr; ++d) {
            int tf = t.fast_tmax - d;  // sigma <= floor((P-1) 2^(2F - 3 - 2t))
            t.fast_thr[d] = Pm1.shift(2 * kSigmaFracBits - 3 - 2 * tf).clamp_u64();
            int ta = t.accu_thi - d;   // X <= floor((P-1) 2^(-1 - 2t))
            t.accu_thr[d] = Pm1.shift(-1 - 2 * ta).clamp_u64();
        }
        t.max_abits_fast = std::max(0, t.fast_tmax + 1);
        t.max_abits_accu = std::max(0, t.accu_thi + kAccuIntBits);

        for (int l = 0; l < n; ++l) {
            ModConst &mc = t.mod[l];
            const uint32_t p = (uint32_t)all[l];
            mc.p = p;
            mc.half = (p + 1) / 2;
            mc.pf = (float)p;
            mc.ipf = 1.0f / (float)p;  // correctly rounded single division
            // residue split: weights of the bytes of a word vector (2^(8 j) mod p, in
            // [0, p - 1]) and the offsets that remove the bias 2^(32 W - 1) and add the
            // 128 that makes every residue a byte in [0, 255]
            uint32_t pw = 1;  // 2^(8 j) mod p
            for (int j = 0; j < 4 * kMaxSplitWords; ++j) {
                mc.wbyte[j / 4] |= pw << (8 * (j % 4));
                pw = (pw * 256u) % p;
            }
            for (int w = 1; w <= kMaxSplitWords; ++w) {
                uint32_t b = 1;  // 2^(32 w - 1) mod p
                for (int e = 0; e < 32 * w - 1; ++e) b = (b * 2u) % p;
                mc.wbias[w - 1] = 128u - b;
            }
            // exact: 128 ipf and 0.5 are multiples of 2^-24 (ipf has 24 bits at exponent -8)
            // and their difference is below 1 in magnitude, so it fits in 24 bits
            mc.rbias = 0.5f - 128.0f * mc.ipf;
            // Step II: q_l = (P/p_l)^-1 mod p_l, s_l = (P/p_l) q_l
            const Big Ml = P.div(p);
            const uint32_t q = inverse_mod(Ml.mod(p), p);
            const Big s = Ml.mul(q);
            for (int c = 0; c < std::min(t.nchunks, kMaxChunks); ++c) mc.schunk[c] = chunk(s, c);
        }
    }
}

}  // namespace ozc
