// Host-side construction of the dictionary form of a CRS matrix (the
// CsrView::code and CsrView::ccode arrays): distinct column offsets,
// distinct values, codes and value tables.  Used for the solver matrices of
// a handle and for the operators of an AMG hierarchy's levels.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "core.h"

namespace mrhs {
namespace dict {

// Distinct keys in order of first appearance, at most `limit`; open
// addressing over a power-of-two table.
template <typename K>
struct KeySet {
    std::vector<K> keys;
    std::vector<int32_t> slot;  // index into keys + 1, 0 empty
    uint64_t mask = 0;
    explicit KeySet(int limit)
    {
        size_t cap = 16;
        while (cap < 4 * static_cast<size_t>(limit))
            cap *= 2;
        slot.assign(cap, 0);
        mask = cap - 1;
    }
    // MurmurHash3's 64-bit finalizer: every key bit reaches the low bits the
    // table uses (values such as 4 + k 2^-10 have zero low mantissa bits)
    static uint64_t hash(K k)
    {
        uint64_t z = static_cast<uint64_t>(k);
        z ^= z >> 33;
        z *= 0xff51afd7ed558ccdull;
        z ^= z >> 33;
        z *= 0xc4ceb9fe1a85ec53ull;
        return z ^ (z >> 33);
    }
    // index of k, inserting it; -1 when that would exceed limit
    int32_t add(K k, int limit)
    {
        for (uint64_t h = hash(k) & mask;; h = (h + 1) & mask) {
            const int32_t e = slot[h];
            if (!e) {
                if (static_cast<int>(keys.size()) >= limit)
                    return -1;
                keys.push_back(k);
                slot[h] = static_cast<int32_t>(keys.size());
                return slot[h] - 1;
            }
            if (keys[e - 1] == k)
                return e - 1;
        }
    }
    int32_t find(K k) const
    {
        for (uint64_t h = hash(k) & mask;; h = (h + 1) & mask) {
            const int32_t e = slot[h];
            if (!e || keys[e - 1] == k)
                return e - 1;
        }
    }
};

inline int threads()
{
    const unsigned hw = std::thread::hardware_concurrency();
    return std::max(1, std::min(16, static_cast<int>(hw ? hw : 1)));
}

// Runs fn(lo, hi, t) over T contiguous row ranges of [0, n) in threads.
template <class F>
void row_ranges(int32_t n, int T, F &&fn)
{
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        const int32_t lo = static_cast<int32_t>(static_cast<int64_t>(n) * t / T);
        const int32_t hi = static_cast<int32_t>(static_cast<int64_t>(n) * (t + 1) / T);
        th.emplace_back([&fn, lo, hi, t] { fn(lo, hi, t); });
    }
    for (auto &x : th)
        x.join();
}

// Distinct keys of key(i, j) over the entries j of rows i in [0, n), in order
// of first appearance in row order, at most limit (false when there are more).
template <typename K, class KeyOf>
bool distinct_keys(int32_t n, const int32_t *rp, int limit, KeyOf key, KeySet<K> &out)
{
    const int T = threads();
    std::vector<KeySet<K>> local(T, KeySet<K>(limit));
    std::vector<char> over(T, 0);
    row_ranges(n, T, [&](int32_t lo, int32_t hi, int t) {
        for (int32_t i = lo; i < hi && !over[t]; ++i)
            for (int32_t j = rp[i]; j < rp[i + 1]; ++j)
                if (local[t].add(key(i, j), limit) < 0) {
                    over[t] = 1;
                    break;
                }
    });
    for (int t = 0; t < T; ++t) {
        if (over[t])
            return false;
        for (K k : local[t].keys)
            if (out.add(k, limit) < 0)
                return false;
    }
    return true;
}

template <typename V>
struct BitsOf;
template <>
struct BitsOf<double> {
    using U = uint64_t;
};
template <>
struct BitsOf<float> {
    using U = uint32_t;
};

// The distinct column offsets col - row of a matrix when there are at most
// kDictOffs of them (ok), with the bits ob of an offset index.
struct Offsets {
    KeySet<int64_t> set{kDictOffs};
    bool ok = false;
    int ob = 0;
};

inline void offsets(int32_t n, const int32_t *rp, const int32_t *ci, Offsets &o)
{
    auto off = [&](int32_t i, int32_t j) { return static_cast<int64_t>(ci[j]) - i; };
    o.ok = distinct_keys<int64_t>(n, rp, kDictOffs, off, o.set);
    o.ob = 0;
    while (o.ok && (1 << o.ob) < static_cast<int>(o.set.keys.size()))
        ++o.ob;
}

// Codes of one value array hv over the entries of a matrix: 16-bit codes
// (value index << ob | offset index, 8 codes of padding) when the offsets
// fit, else 32-bit column codes (value index << cb | column, 4 codes of
// padding) when the columns fit beside the value index; ok = false when the
// array has more than kDictVals distinct values (bit patterns) or neither
// form applies.
template <typename V>
struct Codes {
    bool ok = false;
    std::vector<uint16_t> code;
    std::vector<uint32_t> ccode;
    std::vector<V> tab;
    int cb = 0;
};

template <typename V>
Codes<V> codes(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const V *hv, const Offsets &offs)
{
    using U = typename BitsOf<V>::U;
    Codes<V> out;
    const int limit = offs.ok ? std::min(kDictVals, 1 << (16 - offs.ob)) : kDictVals;
    KeySet<U> vals(limit);
    auto bits = [&](int32_t, int32_t j) {
        U u;
        std::memcpy(&u, &hv[j], sizeof(U));
        return u;
    };
    if (!distinct_keys<U>(n, rp, limit, bits, vals))
        return out;
    if (!offs.ok) {
        int vb = 1;  // at least one bit, so the column field is at most 31 bits
        while ((1 << vb) < static_cast<int>(vals.keys.size()))
            ++vb;
        out.cb = 32 - vb;
        if (static_cast<int64_t>(n) > (static_cast<int64_t>(1) << out.cb))
            return out;
    }
    const size_t ncode = static_cast<size_t>(nnz) + (offs.ok ? 8 : 4);
    if (offs.ok)
        out.code.assign(ncode, 0);
    else
        out.ccode.assign(ncode, 0);
    row_ranges(n, threads(), [&](int32_t lo, int32_t hi, int) {
        for (int32_t i = lo; i < hi; ++i)
            for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
                const uint32_t v = static_cast<uint32_t>(vals.find(bits(i, j)));
                if (offs.ok)
                    out.code[j] = static_cast<uint16_t>((v << offs.ob) |
                                                        offs.set.find(static_cast<int64_t>(ci[j]) - i));
                else
                    out.ccode[j] = (v << out.cb) | static_cast<uint32_t>(ci[j]);
            }
    });
    out.tab.resize(vals.keys.size());
    std::memcpy(out.tab.data(), vals.keys.data(), sizeof(V) * out.tab.size());
    out.ok = true;
    return out;
}

} // namespace dict
} // namespace mrhs
