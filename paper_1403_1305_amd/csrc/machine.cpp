// machine.cpp -- host construction of the goto / failure / output functions and
// their full-DFA form (see machine.h).
#include "machine.h"

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstring>
#include <thread>

#include "../../include/ac.h"

namespace acm {
namespace {

// f(begin, end) over [0, n) split into contiguous ranges, one per thread
// (the caller's thread takes the first). Ranges are disjoint, so workers that
// write only their own indices need no synchronisation.
template <typename F>
void parallel_for(uint32_t threads, size_t n, const F &f) {
    constexpr size_t kGrain = 2048;
    const size_t T = std::min<size_t>(std::max<uint32_t>(1, threads), (n + kGrain - 1) / kGrain);
    if (T <= 1) {
        f(size_t(0), n);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve(T - 1);
    for (size_t t = 1; t < T; ++t) pool.emplace_back([&f, n, t, T] { f(n * t / T, n * (t + 1) / T); });
    f(size_t(0), n / T);
    for (std::thread &th : pool) th.join();
}

uint32_t build_threads(uint32_t want) {
    if (want) return std::min<uint32_t>(want, 64);
    const uint32_t hw = std::thread::hardware_concurrency();
    return std::max<uint32_t>(1, std::min<uint32_t>(hw ? hw : 1, 16));
}

uint32_t ceil_log2(uint32_t x) {
    uint32_t k = 0;
    while ((1u << k) < x) ++k;
    return k;
}

// Byte classes. Bytes that occur in some pattern get a column; all others
// send every state back to the root (no pattern can continue through them).
// When the pattern alphabet has at most 8 letters and some window of <= 3
// consecutive bits tells them apart, the column is that bit field, which the
// scan kernels compute with a shift and a mask instead of a table lookup.
void assign_classes(const bool present[256], Machine &m) {
    uint32_t sigma = 0;
    for (int b = 0; b < 256; ++b) sigma += present[b];
    m.sigma = sigma;
    std::memset(m.cmap, kNoClass, sizeof(m.cmap));
    if (sigma <= 8) {
        for (uint32_t k = ceil_log2(sigma); k <= 3 && !m.hashed; ++k) {
            for (uint32_t sh = 0; sh + k <= 8 && !m.hashed; ++sh) {
                uint32_t seen = 0;
                bool ok = true;
                for (int b = 0; b < 256 && ok; ++b) {
                    if (!present[b]) continue;
                    uint32_t h = (uint32_t(b) >> sh) & ((1u << k) - 1);
                    ok = !(seen & (1u << h));
                    seen |= 1u << h;
                }
                if (!ok) continue;
                m.hashed = true;
                m.hash_shift = sh;
                m.n_cols = 1u << k;
                for (uint32_t h = 0; h < 8; ++h) {
                    // a byte that hashes to column h can never equal a letter owned
                    // by another column; unused columns get such a byte
                    m.hash_letter[h] = uint8_t(((h ^ 1u) & ((1u << k) - 1)) << sh);
                    if (k == 0) m.hash_letter[h] = 0;
                }
                for (int b = 0; b < 256; ++b)
                    if (present[b]) {
                        uint32_t h = (uint32_t(b) >> sh) & ((1u << k) - 1);
                        m.cmap[b] = uint8_t(h);
                        m.hash_letter[h] = uint8_t(b);
                    }
            }
        }
    }
    if (!m.hashed) {
        m.n_cols = sigma;
        uint32_t r = 0;
        for (int b = 0; b < 256; ++b)
            if (present[b]) m.cmap[b] = uint8_t(r++);
    }
    m.cols_pow2 = (m.n_cols & (m.n_cols - 1)) == 0;
    m.log2_cols = m.cols_pow2 ? ceil_log2(m.n_cols) : 0;
}

// Depth-first walk of the goto function below node x (depth d, window code
// `code` so far) that fills the start-position gate: the windows whose class
// string runs through x and then leaves the trie (or x at depth kGateQ)
// stop at x. `path` holds the patterns ending on the path to x's parent;
// `lists` receives (node, pattern) for every node with a non-empty path.
void gate_visit(Machine &m, uint32_t x, uint32_t d, uint32_t code, std::vector<uint32_t> &path,
                std::vector<std::pair<uint32_t, uint32_t>> &lists) {
    const size_t mark = path.size();
    for (uint32_t k = m.own_off[x]; k < m.own_off[x + 1]; ++k) path.push_back(m.own_ids[k]);
    for (uint32_t id : path) lists.emplace_back(x, id);
    const uint32_t entry = x | d << kGateNodeBits | (path.empty() ? 0u : kGatePathFlag);
    if (d == kGateQ) {
        // a pattern of kGateQ bytes or more begins with this window
        m.gate_node[code] = entry;
        m.gate_bits[code >> 5] |= 1u << (code & 31);
    } else {
        for (uint32_t c = 0; c < 4; ++c) {
            const uint32_t cc = code | c << (2 * d);
            const uint32_t g = m.go[size_t(x) * 4 + c];
            if (g) {
                gate_visit(m, g & kStateMask, d + 1, cc, path, lists);
                continue;
            }
            // no edge: every window with this prefix stops at x, and can
            // begin only the patterns that end on the path to x
            const uint32_t span = 1u << (2 * (kGateQ - d - 1));
            for (uint32_t e = 0; e < span; ++e) {
                const uint32_t w = cc | e << (2 * (d + 1));
                m.gate_node[w] = entry;
                if (!path.empty()) m.gate_bits[w >> 5] |= 1u << (w & 31);
            }
        }
    }
    path.resize(mark);
}

// The start-position gate of a 4-column machine with bit-field classes (see
// Machine::gate_bits), from the goto function and own outputs in final ids.
void build_gate(Machine &m, const uint8_t *pat, const uint64_t *off) {
    const uint32_t S = m.n_states, n = m.n_patterns;
    m.pat_len.resize(n);
    for (uint32_t k = 0; k < n; ++k) m.pat_len[k] = uint32_t(off[k + 1] - off[k]);
    m.gate_bits.assign(kGateCodes / 32, 0u);
    m.gate_node.assign(kGateCodes, 0u);
    std::vector<uint32_t> path;
    std::vector<std::pair<uint32_t, uint32_t>> lists;
    gate_visit(m, 0, 0, 0, path, lists);
    m.path_off.assign(size_t(S) + 1, 0u);
    for (auto &e : lists) m.path_off[e.first + 1]++;
    for (uint32_t s = 0; s < S; ++s) m.path_off[s + 1] += m.path_off[s];
    m.path_ids.assign(lists.size(), 0u);
    {
        std::vector<uint32_t> fill(m.path_off.begin(), m.path_off.end() - 1);
        for (auto &e : lists) m.path_ids[fill[e.first]++] = e.second;
    }
    for (uint32_t s = 0; s < S; ++s)
        std::sort(m.path_ids.begin() + m.path_off[s], m.path_ids.begin() + m.path_off[s + 1]);
    m.path_one.assign(S, kOneMany);
    for (uint32_t s = 0; s < S; ++s)
        if (m.path_off[s + 1] - m.path_off[s] == 1) {
            const uint32_t id = m.path_ids[m.path_off[s]];
            if (id < (1u << 28)) m.path_one[s] = id | m.pat_len[id] << 28;  // lengths on a path are <= kGateQ
        }
    uint64_t set = 0;
    for (uint32_t w : m.gate_bits) set += uint32_t(__builtin_popcount(w));
    m.gate_pass = double(set) / double(kGateCodes);
    // second level: the class strings of kGateQ2 bytes patterns begin with
    m.gate2_bits.assign(kGate2Bits / 32, 0u);
    uint64_t work = 0;  // class strings to hash: every extension of the short patterns
    for (uint32_t k = 0; k < n; ++k)
        work += m.pat_len[k] >= kGateQ2 ? 1ull : 1ull << (2 * (kGateQ2 - m.pat_len[k]));
    if (work > 8ull * kGate2Bits) {
        // so many short patterns that the level would pass nearly everything
        std::fill(m.gate2_bits.begin(), m.gate2_bits.end(), ~0u);
        return;
    }
    for (uint32_t k = 0; k < n; ++k) {
        const uint64_t len = off[k + 1] - off[k];
        const uint32_t L = uint32_t(std::min<uint64_t>(len, kGateQ2));
        uint32_t code = 0;
        for (uint32_t i = 0; i < L; ++i) code |= uint32_t(m.cmap[pat[off[k] + i]]) << (2 * i);
        const uint32_t span = 1u << (2 * (kGateQ2 - L));
        for (uint32_t e = 0; e < span; ++e) {
            const uint32_t y = code | (L < kGateQ2 ? e << (2 * L) : 0u);
            const uint32_t h = gate2_hash(y), h2 = gate2_hash2(y);
            m.gate2_bits[h >> 5] |= 1u << (h & 31);
            m.gate2_bits[h2 >> 5] |= 1u << (h2 & 31);
        }
    }
}

// The hashed start-position gate (see Machine::qg_bits), from the goto
// function; every pattern is at least kQgQ bytes long.
void build_qgate(Machine &m, const uint8_t *pat, const uint64_t *off) {
    const uint32_t n = m.n_patterns, C = m.n_cols;
    struct Win {
        uint32_t x, y, node;
    };
    std::vector<Win> wins;
    wins.reserve(n);
    std::vector<uint64_t> freq(256, 0);
    uint64_t total = 0;
    for (uint32_t k = 0; k < n; ++k) {
        const uint8_t *p = pat + off[k];
        for (uint64_t i = 0; i < off[k + 1] - off[k]; ++i) ++freq[p[i]];
        total += off[k + 1] - off[k];
        uint32_t x = 0;
        for (uint32_t d = 0; d < kQgQ; ++d) x = m.go[size_t(x) * C + m.cmap[p[d]]] & kStateMask;
        wins.push_back({uint32_t(p[0]) | uint32_t(p[1]) << 8 | uint32_t(p[2]) << 16,
                        uint32_t(p[3]) | uint32_t(p[4]) << 8 | uint32_t(p[5]) << 16, x});
    }
    std::sort(wins.begin(), wins.end(), [](const Win &a, const Win &b) { return a.x != b.x ? a.x < b.x : a.y < b.y; });
    wins.erase(std::unique(wins.begin(), wins.end(), [](const Win &a, const Win &b) { return a.x == b.x && a.y == b.y; }),
               wins.end());
    m.qg_bits.assign(kQgWords, 0u);
    double cover = 0.0;
    for (const Win &w : wins) {
        const uint32_t h = qg_hash(w.x, w.y);
        m.qg_bits[qg_word(h)] |= qg_mask(h);
        double pr = 1.0;
        for (uint32_t d = 0; d < 3; ++d)
            pr *= double(freq[(w.x >> (8 * d)) & 0xffu]) * double(freq[(w.y >> (8 * d)) & 0xffu]) /
                  (double(total) * double(total));
        cover += pr;
    }
    // the window table: cuckoo hashing with two slot choices, at most 40% full;
    // a table where some insertion finds no place is rebuilt twice as large
    uint32_t bits = 8;
    while ((1ull << bits) * 2 < 5ull * wins.size()) ++bits;
    for (;; ++bits) {
        const uint32_t shift = 32 - bits;
        std::vector<int32_t> at(size_t(1) << bits, -1);  // slot -> window index
        bool ok = true;
        for (uint32_t k = 0; k < wins.size() && ok; ++k) {
            uint32_t cur = k;
            uint32_t slot = qg_slot_a(wins[cur].x, wins[cur].y) >> shift;
            for (uint32_t kick = 0;; ++kick) {
                if (at[slot] < 0) {
                    at[slot] = int32_t(cur);
                    break;
                }
                const uint32_t alt = qg_slot_b(wins[cur].x, wins[cur].y) >> shift;
                if (slot != alt && at[alt] < 0) {
                    at[alt] = int32_t(cur);
                    break;
                }
                if (kick == 500) {
                    ok = false;
                    break;
                }
                // take the slot and move its window to the other of its two
                std::swap(cur, reinterpret_cast<uint32_t &>(at[slot]));
                const uint32_t a = qg_slot_a(wins[cur].x, wins[cur].y) >> shift;
                slot = a == slot ? qg_slot_b(wins[cur].x, wins[cur].y) >> shift : a;
            }
        }
        if (!ok) continue;
        m.qg_tab_bits = bits;
        m.qg_tab.assign(size_t(4) << bits, 0u);
        for (size_t s = 0; s < at.size(); ++s) {
            if (at[s] < 0) continue;
            const Win &w = wins[size_t(at[s])];
            uint32_t *e = &m.qg_tab[s * 4];
            e[0] = w.x | (w.y & 0xffu) << 24;
            e[1] = w.y >> 8 | kQgUsed | (m.own_off[w.node + 1] > m.own_off[w.node] ? kQgOwn : 0u);
            e[2] = w.node;
            uint32_t kids = C > 32 ? ~0u : 0u;
            for (uint32_t c = 0; c < C && C <= 32; ++c)
                if (m.go[size_t(w.node) * C + c]) kids |= 1u << c;
            e[3] = kids;
        }
        break;
    }
    // a window that begins no pattern passes when both of its bits are set:
    // about the mean over words of (set bits / 32)^2
    double fp = 0.0;
    for (uint32_t w : m.qg_bits) {
        const double f = double(__builtin_popcount(w)) / 32.0;
        fp += f * f;
    }
    fp /= double(kQgWords);
    m.gate_pass = std::min(1.0, cover + (1.0 - std::min(1.0, cover)) * fp);
}

}  // namespace

int build_machine(const uint8_t *pat, const uint64_t *off, uint32_t n, const HotPlan &plan,
                  Machine &m, std::string &err) {
    auto t0 = std::chrono::steady_clock::now();
    if (n == 0 || pat == nullptr || off == nullptr) {
        err = "ac_build: need at least one pattern and non-null pattern arrays";
        return AC_ERR_INVALID;
    }
    uint64_t total = 0;
    bool present[256] = {false};
    m.n_patterns = n;
    m.m_max = 0;
    for (uint32_t k = 0; k < n; ++k) {
        if (off[k + 1] <= off[k]) {
            err = "ac_build: pattern " + std::to_string(k) + " is empty or its offsets decrease";
            return AC_ERR_INVALID;
        }
        uint64_t len = off[k + 1] - off[k];
        if (len >= (1ull << 31)) {
            err = "ac_build: pattern longer than 2^31 bytes";
            return AC_ERR_TOO_LARGE;
        }
        total += len;
        m.m_max = std::max<uint32_t>(m.m_max, uint32_t(len));
        for (uint64_t i = off[k]; i < off[k + 1]; ++i) present[pat[i]] = true;
    }
    if (total + 1 >= (1ull << 31)) {
        err = "ac_build: more than 2^31 pattern bytes";
        return AC_ERR_TOO_LARGE;
    }
    assign_classes(present, m);
    const uint32_t C = m.n_cols;

    // ---- goto function: a trie, nodes numbered as they are created
    std::vector<int32_t> kid;  // node * C + c -> node, -1 if no edge
    kid.reserve(size_t(std::min<uint64_t>(total + 1, 1u << 24)) * C);
    kid.assign(C, -1);
    uint32_t nodes = 1;
    std::vector<std::pair<uint32_t, uint32_t>> ends;  // (node, pattern id)
    ends.reserve(n);
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t v = 0;
        for (uint64_t i = off[k]; i < off[k + 1]; ++i) {
            uint32_t c = m.cmap[pat[i]];
            int32_t w = kid[size_t(v) * C + c];
            if (w < 0) {
                w = int32_t(nodes++);
                kid[size_t(v) * C + c] = w;
                kid.resize(size_t(nodes) * C, -1);
            }
            v = uint32_t(w);
        }
        ends.emplace_back(v, k);
    }
    const uint32_t S = nodes;
    if (uint64_t(S) * C >= (1ull << 31)) {
        err = "ac_build: transition table would exceed 2^31 entries";
        return AC_ERR_TOO_LARGE;
    }

    // ---- breadth-first order (children visited by column), one level at a
    // time: count each node's children, prefix-sum, then place them
    const uint32_t NT = build_threads(plan.threads);
    std::vector<uint32_t> order(S), bfs(S);
    std::vector<uint32_t> level{0, 1};  // level d holds breadth-first ids [level[d], level[d+1])
    order[0] = 0;
    bfs[0] = 0;
    {
        std::vector<uint32_t> cnt;
        size_t lo = 0, hi = 1;
        while (lo < hi) {
            const size_t nl = hi - lo;
            cnt.assign(nl + 1, 0);
            parallel_for(NT, nl, [&](size_t b, size_t e) {
                for (size_t i = b; i < e; ++i) {
                    const int32_t *row = &kid[size_t(order[lo + i]) * C];
                    uint32_t k = 0;
                    for (uint32_t c = 0; c < C; ++c) k += row[c] >= 0;
                    cnt[i + 1] = k;
                }
            });
            for (size_t i = 0; i < nl; ++i) cnt[i + 1] += cnt[i];
            parallel_for(NT, nl, [&](size_t b, size_t e) {
                for (size_t i = b; i < e; ++i) {
                    const int32_t *row = &kid[size_t(order[lo + i]) * C];
                    size_t q = hi + cnt[i];
                    for (uint32_t c = 0; c < C; ++c)
                        if (row[c] >= 0) {
                            order[q] = uint32_t(row[c]);
                            bfs[row[c]] = uint32_t(q);
                            ++q;
                        }
                }
            });
            lo = hi;
            hi += cnt[nl];
            if (hi > lo) level.push_back(uint32_t(hi));
        }
    }
    // children in breadth-first ids
    std::vector<int32_t> child(size_t(S) * C);
    parallel_for(NT, S, [&](size_t b, size_t e) {
        for (size_t i = b; i < e; ++i) {
            const int32_t *row = &kid[size_t(order[i]) * C];
            for (uint32_t c = 0; c < C; ++c) child[i * C + c] = row[c] >= 0 ? int32_t(bfs[row[c]]) : -1;
        }
    });
    std::vector<int32_t>().swap(kid);

    // ---- failure function and full DFA, row by row in breadth-first order.
    // A row only reads the row of its failure state, which is shallower and
    // therefore already final.
    const bool full = !plan.goto_only;
    m.goto_only = plan.goto_only;
    std::vector<uint32_t> delta(full ? size_t(S) * C : 0);
    std::vector<uint32_t> fail(full ? S : 0, 0);
    for (uint32_t c = 0; c < C && full; ++c) {
        int32_t w = child[c];
        delta[c] = w >= 0 ? uint32_t(w) : 0u;
        if (w >= 0) fail[w] = 0;
    }
    // deeper levels in turn; the rows of one level only read shallower rows
    for (size_t d = 1; full && d + 1 < level.size(); ++d) {
        parallel_for(NT, level[d + 1] - level[d], [&](size_t b0, size_t e0) {
            for (size_t b = level[d] + b0; b < level[d] + e0; ++b) {
                const uint32_t *frow = &delta[size_t(fail[b]) * C];
                uint32_t *row = &delta[b * C];
                for (uint32_t c = 0; c < C; ++c) {
                    const int32_t w = child[b * C + c];
                    if (w >= 0) {
                        row[c] = uint32_t(w);
                        fail[w] = frow[c];
                    } else {
                        row[c] = frow[c];
                    }
                }
            }
        });
    }

    // ---- output function: own patterns, plus the failure state's outputs
    std::vector<uint32_t> own_cnt(S + 1, 0);
    for (auto &e : ends) own_cnt[bfs[e.first] + 1]++;
    std::vector<uint32_t> own_off(S + 1, 0);
    for (uint32_t b = 0; b < S; ++b) own_off[b + 1] = own_off[b] + own_cnt[b + 1];
    std::vector<uint32_t> own_ids(n);
    {
        std::vector<uint32_t> fill(own_off.begin(), own_off.end() - 1);
        for (auto &e : ends) own_ids[fill[bfs[e.first]]++] = e.second;  // ids ascending per state
    }
    std::vector<uint32_t> out_off(S + 1, 0);
    std::vector<uint32_t> out_ids;
    if (!full) {  // failure-less: a state outputs the patterns ending there
        out_off = own_off;
        out_ids = own_ids;
    } else {
        // a level at a time: sizes, offsets, then the merges (ascending ids)
        out_off[1] = own_off[1] - own_off[0];
        out_ids.assign(own_ids.begin() + own_off[0], own_ids.begin() + own_off[1]);
        for (size_t d = 1; d + 1 < level.size(); ++d) {
            const size_t lo = level[d], hi = level[d + 1];
            parallel_for(NT, hi - lo, [&](size_t b0, size_t e0) {
                for (size_t b = lo + b0; b < lo + e0; ++b)
                    out_off[b + 1] = (own_off[b + 1] - own_off[b]) + (out_off[fail[b] + 1] - out_off[fail[b]]);
            });
            uint64_t at = out_off[lo];
            for (size_t b = lo; b < hi; ++b) {
                at += out_off[b + 1];
                if (at >= (1ull << 32) - 1) {
                    err = "ac_build: output sets exceed 2^32 entries";
                    return AC_ERR_TOO_LARGE;
                }
                out_off[b + 1] = uint32_t(at);
            }
            out_ids.resize(at);
            parallel_for(NT, hi - lo, [&](size_t b0, size_t e0) {
                for (size_t b = lo + b0; b < lo + e0; ++b) {
                    const uint32_t f = fail[b];
                    std::merge(own_ids.begin() + own_off[b], own_ids.begin() + own_off[b + 1],
                               out_ids.begin() + out_off[f], out_ids.begin() + out_off[f + 1],
                               out_ids.begin() + out_off[b]);
                }
            });
        }
    }
    auto accepts = [&](uint32_t b) { return out_off[b + 1] > out_off[b]; };

    // ---- final numbering, in ranges:
    //   [0, H)                 hot: non-final states whose rows form the 16-bit
    //                          LDS image, the shallowest first (breadth-first
    //                          order approximates visit frequency on text
    //                          unrelated to the patterns); the root is 0;
    //   [H, term_end)          final states where some pattern ends exactly;
    //   [term_end, acc_end)    final states whose outputs all come by failure;
    //   [acc_end, S)           the other non-final states, those that a hot row
    //                          leads to first.
    // A step into a state >= H is then the one event the scan kernels must
    // look at, and "final" and "pattern ends here" are range tests. Every
    // successor of a hot row must fit the 16-bit entries: the image shrinks
    // until it does (or is dropped if the final states alone do not fit).
    uint32_t hot_budget = 0;
    // (the image kernels address the 32-bit table with 32-bit byte offsets)
    if (plan.lds_bytes > 256 && uint64_t(S) * C * 4ull < (1ull << 32)) {
        const bool full_fits = 256ull + uint64_t(S) * C * 4ull <= plan.lds_bytes;
        if (!(plan.only_if_needed && full_fits)) {
            hot_budget = (plan.lds_bytes - 256) / (2 * C);
            if (plan.max_states) hot_budget = std::min(hot_budget, plan.max_states);
        }
    }
    auto terminal = [&](uint32_t b) { return own_off[b + 1] > own_off[b]; };
    uint32_t A = 0, T = 0;
    for (uint32_t b = 0; b < S; ++b) {
        A += accepts(b);
        T += terminal(b);
    }
    std::vector<uint32_t> cand;  // non-final states in breadth-first order (the root first)
    const uint32_t want = std::max<uint32_t>(1, std::min<uint32_t>(hot_budget, kHotIdLimit));
    for (uint32_t b = 0; b < S && cand.size() < want; ++b)
        if (!accepts(b)) cand.push_back(b);
    uint32_t H = uint32_t(cand.size());
    std::vector<uint8_t> mark(S, 0);  // 1 = hot, 2 = non-final target of a hot row
    bool image = hot_budget > 0;
    while (true) {
        std::fill(mark.begin(), mark.end(), 0);
        for (uint32_t i = 0; i < H; ++i) mark[cand[i]] = 1;
        uint32_t extra = 0;
        if (image)
            for (uint32_t i = 0; i < H; ++i)
                for (uint32_t c = 0; c < C; ++c) {
                    // a hot row's successors: DFA targets, or goto children
                    // (a goto child is also the DFA target of its column)
                    uint32_t t;
                    if (full) {
                        t = delta[size_t(cand[i]) * C + c];
                    } else {
                        const int32_t w = child[size_t(cand[i]) * C + c];
                        if (w < 0) continue;
                        t = uint32_t(w);
                    }
                    if (!mark[t] && !accepts(t)) {
                        mark[t] = 2;
                        ++extra;
                    }
                }
        if (image && H < kMinHotStates && H < cand.size()) {
            image = false;  // shrunk to too few rows to be worth an LDS image
            H = 1;
            continue;
        }
        if (!image || uint64_t(H) + A + extra <= kHotIdLimit) break;
        if (H == 1 || uint64_t(A) + 1 > kHotIdLimit) {
            image = false;  // the final states alone overflow 16-bit ids
            H = 1;
            continue;
        }
        const uint64_t cut = std::max<uint64_t>(1, (uint64_t(H) + A + extra - kHotIdLimit + 1) / 2);
        H = cut >= H ? 1u : uint32_t(H - cut);
    }
    std::vector<uint32_t> perm(S);  // bfs id -> final id
    {
        uint32_t next = 0;
        for (uint32_t i = 0; i < H; ++i) perm[cand[i]] = next++;
        for (uint32_t b = 0; b < S; ++b)
            if (!mark[b] && terminal(b)) perm[b] = next++;
        for (uint32_t b = 0; b < S; ++b)
            if (!mark[b] && accepts(b) && !terminal(b)) perm[b] = next++;
        for (uint32_t b = 0; b < S; ++b)
            if (mark[b] == 2) perm[b] = next++;
        for (uint32_t b = 0; b < S; ++b)
            if (!mark[b] && !accepts(b)) perm[b] = next++;
    }
    m.term_end = H + T;
    m.acc_end = H + A;
    if (!image) H = 0;  // numbering keeps the root alone in front; no image rows
    std::vector<uint32_t> inv(S);
    for (uint32_t b = 0; b < S; ++b) inv[perm[b]] = b;

    // ---- device tables in final ids
    m.n_states = S;
    m.dfa.assign(full ? size_t(S) * C : 0, 0);
    m.go.assign(size_t(S) * C, 0);
    m.out_off.assign(S + 1, 0);
    m.own_off.assign(S + 1, 0);
    m.out_ids.clear();
    m.out_ids.reserve(out_ids.size());
    m.own_ids.clear();
    m.own_ids.reserve(n);
    parallel_for(NT, S, [&](size_t f0, size_t f1) {
        for (size_t f = f0; f < f1; ++f) {
            const uint32_t b = inv[f];
            for (uint32_t c = 0; c < C; ++c) {
                if (full) {
                    const uint32_t t = delta[size_t(b) * C + c];
                    m.dfa[f * C + c] = perm[t] | (accepts(t) ? kAccept : 0u);
                }
                const int32_t w = child[size_t(b) * C + c];
                if (w >= 0) m.go[f * C + c] = perm[w] | (own_off[w + 1] > own_off[w] ? kAccept : 0u);
            }
        }
    });
    for (uint32_t f = 0; f < S; ++f) {
        const uint32_t b = inv[f];
        m.out_off[f + 1] = m.out_off[f] + (out_off[b + 1] - out_off[b]);
        m.own_off[f + 1] = m.own_off[f] + (own_off[b + 1] - own_off[b]);
    }
    m.out_ids.resize(out_ids.size());
    m.own_ids.resize(n);
    parallel_for(NT, S, [&](size_t f0, size_t f1) {
        for (size_t f = f0; f < f1; ++f) {
            const uint32_t b = inv[f];
            std::copy(out_ids.begin() + out_off[b], out_ids.begin() + out_off[b + 1], m.out_ids.begin() + m.out_off[f]);
            std::copy(own_ids.begin() + own_off[b], own_ids.begin() + own_off[b + 1], m.own_ids.begin() + m.own_off[f]);
        }
    });
    m.hot_states = H;
    m.hot_dfa.assign(full ? size_t(H) * C : 0, 0);
    m.hot_go.assign(size_t(H) * C, 0);
    for (uint32_t f = 0; f < H; ++f)
        for (uint32_t c = 0; c < C; ++c) {
            // successors of hot rows were numbered below kHotIdLimit above
            if (full) m.hot_dfa[size_t(f) * C + c] = uint16_t(m.dfa[size_t(f) * C + c] & kStateMask);
            m.hot_go[size_t(f) * C + c] = uint16_t(m.go[size_t(f) * C + c] & kStateMask);
        }
    // Two bytes per lookup from the states outside the image (on request):
    // half as many dependent global lookups for the walks that leave it.
    m.pair.clear();
    m.pair_states = 0;
    if (plan.pair_rows && full && m.hashed && C == 4 && H > 0 && S - H <= kPairMaxStates) {
        m.pair_states = S - H;
        m.pair.assign(size_t(S - H) * 16, 0);
        parallel_for(NT, S - H, [&](size_t b0, size_t e0) {
            for (size_t i = b0; i < e0; ++i) {
                const size_t s = H + i;
                for (uint32_t c1 = 0; c1 < 4; ++c1) {
                    const uint32_t mid = m.dfa[s * 4 + c1];
                    const size_t row = size_t(mid & kStateMask) * 4;
                    for (uint32_t c2 = 0; c2 < 4; ++c2)
                        m.pair[i * 16 + (c1 | c2 << 2)] = (m.dfa[row + c2] & kStateMask) | (mid & kAccept);
                }
            }
        });
    }
    m.gate_bits.clear();
    m.gate2_bits.clear();
    m.gate_node.clear();
    m.path_off.clear();
    m.path_ids.clear();
    m.pat_len.clear();
    m.path_one.clear();
    m.own_one.clear();
    m.qg_bits.clear();
    m.qg_tab.clear();
    m.qg_tab_bits = 0;
    m.gate_pass = 1.0;
    if (plan.gate && m.hashed && C == 4 && S - 1 <= kGateNodeMask) {
        build_gate(m, pat, off);
    } else if (plan.gate) {
        uint64_t shortest = ~0ull;
        for (uint32_t k = 0; k < n; ++k) shortest = std::min<uint64_t>(shortest, off[k + 1] - off[k]);
        if (n > 0 && shortest >= kQgQ) build_qgate(m, pat, off);
    }
    m.match_rate = 0.0;
    if (!m.gate_bits.empty() || !m.qg_bits.empty()) {
        std::vector<double> lf(256, 0.0);  // log byte frequency over the pattern bytes
        {
            std::vector<uint64_t> cnt(256, 0);
            for (uint64_t i = off[0]; i < off[n]; ++i) ++cnt[pat[i]];
            for (int b = 0; b < 256; ++b)
                if (cnt[b]) lf[b] = std::log(double(cnt[b]) / double(off[n] - off[0]));
        }
        for (uint32_t k = 0; k < n; ++k) {
            double lp = 0.0;
            for (uint64_t i = off[k]; i < off[k + 1] && lp > -80.0; ++i) lp += lf[pat[i]];
            m.match_rate += std::exp(lp);
        }
        m.own_one.assign(S, kOneMany);
        for (uint32_t s = 0; s < S; ++s)
            if (m.own_off[s + 1] - m.own_off[s] == 1) m.own_one[s] = m.own_ids[m.own_off[s]];
    }
    // 16-bit images are copied as 32-bit words: pad them to whole words
    if (m.hot_dfa.size() & 1) m.hot_dfa.push_back(0);
    if (m.hot_go.size() & 1) m.hot_go.push_back(0);
    m.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return AC_OK;
}

}  // namespace acm
