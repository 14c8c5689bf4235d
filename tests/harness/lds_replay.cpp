// Host replay of the counting kernel's LDS index expressions, with a bounds check on every
// access.  TEST INFRASTRUCTURE: it models, for the per-vertex variant of the bit-row
// kernel (one team per root, persistent schedule without splits), the team's LDS arrays
// with the kernel's capacities and row stride, and walks every work item of a directed
// graph the way the team's waves do: staging of S, the member bitmap / hash and filter,
// the second-level list stream (list table cursor), the bit rows, the pair ring and the
// bit-row recursion with its per-vertex counters.  Lanes run one after another; an access
// outside its array aborts with the array, the index and the item.  The replay also
// returns the total and per-vertex counts it computes, so that its model of the
// arithmetic can be checked against the oracle.
//
// Build: g++ -O2 -std=c++17 -shared -fPIC lds_replay.cpp -o liblds_replay.so
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

namespace {

const char *g_item = "";
long g_root = -1;

template <class T>
struct Arr {
    const char *name;
    std::vector<T> v;
    Arr(const char *nm, long n) : name(nm), v((size_t)(n > 0 ? n : 1)) {}
    T &operator[](long i) {
        if (i < 0 || i >= (long)v.size()) {
            fprintf(stderr, "LDS replay: %s[%ld] outside [0, %zu) at root %ld (%s)\n", name, i, v.size(), g_root,
                    g_item);
            abort();
        }
        return v[(size_t)i];
    }
};

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

int popc(uint32_t x) { return __builtin_popcount(x); }

uint32_t gtmask(int z, int w) {
    int zw = z >> 5, zb = z & 31;
    uint32_t hi = zb == 31 ? 0u : (~0u << (zb + 1));
    return w < zw ? 0u : (w > zw ? ~0u : hi);
}

struct Team {
    // capacities as the kernel's TeamLds<W, PV = true, TW> and TierCfg<W, true, LMAX>
    int W, TW, D, Q, RS, HS, HB, SPAN, SW, RING;
    Arr<int32_t> S;
    Arr<uint64_t> H;
    Arr<uint32_t> bm;
    Arr<uint16_t> pre;
    Arr<uint32_t> flt;
    Arr<uint32_t> rows;
    Arr<uint64_t> cnt;
    Arr<uint32_t> ring;     // [TW][RING]
    Arr<int64_t> lt_end, lt_delta;
    Arr<int32_t> lt_row;    // [TW][64]
    Team(int W_)
        : W(W_), TW(W_ == 2 ? 1 : (W_ <= 8 ? 4 : 8)), D(32 * W_), Q(W_ >= 16 ? 4 : 1),
          RS((W_ / Q) % 2 == 1 ? W_ : W_ + Q), HS(pow2_at_least(D <= 128 ? 4 * D : 2 * D)), HB(__builtin_ctz(HS)),
          SPAN(W_ == 2 ? 0 : (W_ == 4 ? 1 << 16 : (W_ <= 16 ? 1 << 15 : 1 << 14))), SW(SPAN > 0 ? SPAN / 32 : 1),
          RING(pow2_at_least(D + 64)), S("S", D), H("H", HS), bm("bm", SW), pre("pre", SW),
          flt("flt", 64), rows("rows", (long)D * RS), cnt("cnt", D), ring("ring", (long)TW * RING),
          lt_end("lt", (long)TW * 64), lt_delta("lt", (long)TW * 64), lt_row("lt", (long)TW * 64) {}
};

struct Graph {
    int64_t n;
    const int64_t *off;
    const int32_t *idx;
    int64_t m;
};

uint32_t hslot(uint32_t key, int hb) { return (key * 2654435761u) >> (32 - hb); }
uint32_t filter_hash(int32_t w) { return ((uint32_t)w * 2246822519u) >> 21; }

int member_find(Team &T, int32_t w, int32_t first, int32_t last, bool bmode) {
    if ((uint32_t)(w - first) > (uint32_t)(last - first)) return -1;
    if (T.SPAN > 0 && bmode) {
        const uint32_t o = (uint32_t)(w - first);
        const uint32_t word = T.bm[o >> 5];
        const uint32_t bit = o & 31u;
        if (!((word >> bit) & 1u)) return -1;
        return (int)T.pre[o >> 5] + popc(word & ((1u << bit) - 1u));
    }
    uint32_t s = hslot((uint32_t)w, T.HB);
    for (int probes = 0;; ++probes) {
        if (probes > T.HS) { fprintf(stderr, "LDS replay: hash probe did not end\n"); abort(); }
        uint64_t e = T.H[s];
        if (e == ~0ull) return -1;
        if ((uint32_t)e == (uint32_t)w) return (int)(e >> 32);
        s = (s + 1) & (T.HS - 1);
    }
}

void load_row(Team &T, int d, int z, std::vector<uint32_t> &r) {
    if (z < 0 || z >= d) {
        fprintf(stderr, "LDS replay: row %d of a set of %d at root %ld\n", z, d, g_root);
        abort();
    }
    for (int q = 0; q < T.W; ++q) r[q] = T.rows[(long)z * T.RS + q];
}

// dfs of the kernel (per-vertex mode): L-cliques inside J; members credited through cnt
uint64_t dfs(Team &T, int d, const std::vector<uint32_t> &J, int L) {
    uint64_t out = 0;
    std::vector<uint32_t> R(J), rz(T.W), K(T.W);
    while (true) {
        int z = -1;
        for (int w = 0; w < T.W; ++w)
            if (z < 0 && R[w]) {
                z = w * 32 + __builtin_ctz(R[w]);
                R[w] &= R[w] - 1;
            }
        if (z < 0) break;
        load_row(T, d, z, rz);
        if (L == 2) {
            unsigned a = 0, c = 0;
            for (int w = 0; w < T.W; ++w) {
                uint32_t t = J[w] & rz[w];
                a += popc(t);
                c += popc(t & gtmask(z, w));
            }
            if (a) T.cnt[z] += a;
            out += c;
        } else {
            for (int w = 0; w < T.W; ++w) K[w] = R[w] & rz[w];
            uint64_t sub = dfs(T, d, K, L - 1);
            if (sub) T.cnt[z] += sub;
            out += sub;
        }
    }
    return out;
}

uint64_t do_pair(Team &T, int d, int x, int y, int need) {
    std::vector<uint32_t> rx(T.W), ry(T.W), J(T.W);
    load_row(T, d, x, rx);
    load_row(T, d, y, ry);
    if (need == 1) {
        unsigned a = 0, c = 0;
        for (int w = 0; w < T.W; ++w) {
            uint32_t t = rx[w] & ry[w];
            a += popc(t & gtmask(x, w));
            c += popc(t & gtmask(y, w));
        }
        if (a) T.cnt[y] += a;
        if (c) T.cnt[x] += c;
        return c;
    }
    for (int w = 0; w < T.W; ++w) J[w] = rx[w] & ry[w] & gtmask(y, w);
    uint64_t sub = dfs(T, d, J, need);
    if (sub) {
        T.cnt[x] += sub;
        T.cnt[y] += sub;
    }
    return sub;
}

// The 64-tier at k >= 7 deals triples (x, y, z) through a second ring kept in the hash
// table's LDS (512 entries): a round of 64 pairs pushes its children in lane order, as much
// as fits, and the lanes take the ring's entries 64 at a time.
struct Ring3 {
    Arr<uint32_t> r;
    unsigned head = 0, tail = 0;
    Ring3() : r("ring3 (hash table)", 512) {}
};

uint64_t take3(Team &T, int d, uint32_t e, int pneed) {
    const int x = (int)(e & 63u), y = (int)((e >> 6) & 63u), z = (int)(e >> 12);
    if (x >= d || y >= d || z >= d || !(x < y && y < z)) { fprintf(stderr, "LDS replay: bad triple\n"); abort(); }
    std::vector<uint32_t> rx(T.W), ry(T.W), rz(T.W), K(T.W);
    load_row(T, d, x, rx);
    load_row(T, d, y, ry);
    load_row(T, d, z, rz);
    for (int w = 0; w < T.W; ++w) K[w] = rx[w] & ry[w] & rz[w] & gtmask(z, w);
    const uint64_t sub = dfs(T, d, K, pneed - 1);
    if (sub) {
        T.cnt[x] += sub;
        T.cnt[y] += sub;
        T.cnt[z] += sub;
    }
    return sub;
}

// one round: lanes 0..nvalid-1 hold the pairs p[lane] (row << 16 | member)
uint64_t deal3(Team &T, int d, Ring3 &q, const uint32_t *p, int nvalid, int pneed) {
    uint64_t out = 0;
    uint64_t R[64];
    uint32_t base[64];
    for (int l = 0; l < 64; ++l) {
        R[l] = 0;
        base[l] = 0;
        if (l < nvalid) {
            const int py = (int)(p[l] >> 16), px = (int)(p[l] & 0xffffu);
            std::vector<uint32_t> rx(T.W), ry(T.W);
            load_row(T, d, px, rx);
            load_row(T, d, py, ry);
            const uint64_t jx = (uint64_t)rx[0] | ((uint64_t)rx[1] << 32), jy = (uint64_t)ry[0] | ((uint64_t)ry[1] << 32);
            const int hi = py > px ? py : px;
            R[l] = jx & jy & ~((2ull << hi) - 1ull);
            base[l] = (uint32_t)px | ((uint32_t)py << 6);
        }
    }
    while (true) {
        unsigned pre[64], c[64], total = 0;
        for (int l = 0; l < 64; ++l) {
            c[l] = (unsigned)__builtin_popcountll(R[l]);
            total += c[l];
            pre[l] = total;
        }
        if (total == 0) break;
        const unsigned space = 512 - (q.tail - q.head);
        for (int l = 0; l < 64; ++l) {
            const unsigned start = pre[l] - c[l];
            unsigned cnt = start >= space ? 0u : (c[l] < space - start ? c[l] : space - start);
            unsigned pos = q.tail + start;
            while (cnt) {
                const int z = __builtin_ctzll(R[l]);
                R[l] &= R[l] - 1;
                q.r[pos & 511u] = base[l] | ((uint32_t)z << 12);
                ++pos;
                --cnt;
            }
        }
        q.tail += total < space ? total : space;
        if (q.tail - q.head > 512u) { fprintf(stderr, "LDS replay: ring3 overrun\n"); abort(); }
        while (q.tail - q.head >= 64) {
            for (int l = 0; l < 64; ++l) out += take3(T, d, q.r[(q.head + l) & 511u], pneed);
            q.head += 64;
        }
    }
    return out;
}

// one root item, per-vertex mode; returns the item's count and adds to pv
uint64_t process_root(Team &T, const Graph &g, int k, int32_t root, int span_max, uint64_t *pv) {
    g_root = root;
    g_item = "stage";
    const int64_t s0 = g.off[root];
    const int64_t dd = g.off[root + 1] - s0;
    if (dd > T.D) { fprintf(stderr, "LDS replay: root %d too large for the tier\n", root); abort(); }
    const int d = (int)dd;
    for (int i = 0; i < d; ++i) T.S[i] = g.idx[s0 + i];
    const int need = k - 1;
    if (d < need || d == 0) return 0;
    const int32_t first = T.S[0], last = T.S[d - 1];
    bool bmode = false;
    if (T.SPAN > 0) bmode = (int64_t)last - (int64_t)first < (int64_t)(T.SPAN < span_max ? T.SPAN : span_max);
    if (bmode) {
        const int nw = ((last - first) >> 5) + 1;
        for (int i = 0; i < nw; ++i) T.bm[i] = 0u;
    } else {
        for (int i = 0; i < T.HS; ++i) T.H[i] = ~0ull;
    }
    if (!bmode)
        for (int i = 0; i < 64; ++i) T.flt[i] = 0u;
    if (need >= 3)
        for (long i = 0; i < (long)d * T.RS; ++i) T.rows[i] = 0u;
    for (int i = 0; i < d; ++i) T.cnt[i] = 0;
    if (bmode) {
        for (int i = 0; i < d; ++i) {
            const uint32_t o = (uint32_t)(T.S[i] - first);
            T.bm[o >> 5] |= 1u << (o & 31u);
            if (i == 0 || ((uint32_t)(T.S[i - 1] - first) >> 5) != (o >> 5)) T.pre[o >> 5] = (uint16_t)i;
        }
    } else {
        for (int i = 0; i < d; ++i) {
            uint32_t s = hslot((uint32_t)T.S[i], T.HB);
            const uint64_t e = ((uint64_t)(uint32_t)i << 32) | (uint32_t)T.S[i];
            for (int probes = 0;; ++probes) {
                if (probes > T.HS) { fprintf(stderr, "LDS replay: hash full\n"); abort(); }
                if (T.H[s] == ~0ull) { T.H[s] = e; break; }
                s = (s + 1) & (T.HS - 1);
            }
        }
    }
    if (!bmode)
        for (int i = 0; i < d; ++i) {
            const uint32_t h = filter_hash(T.S[i]);
            T.flt[h >> 5] |= 1u << (h & 31u);
        }
    uint64_t mine = 0;
    if (need == 1) {
        mine = (uint64_t)d;
        for (int i = 0; i < d; ++i) T.cnt[i] = 1;
    } else {
        g_item = "second level";
        // every wave wv takes the lists S[wv], S[wv + TW], ... 64 at a time
        for (int wv = 0; wv < T.TW; ++wv) {
            const int nl = wv < d ? (d - wv + T.TW - 1) / T.TW : 0;
            for (int gb = 0; gb < nl; gb += 64) {
                int64_t end = 0;
                for (int lane = 0; lane < 64; ++lane) {
                    const int t = gb + lane;
                    int64_t s = 0, e = 0;
                    int row = 0;
                    if (t < nl) {
                        row = wv + T.TW * t;
                        const int32_t u = T.S[row];
                        s = g.off[u];
                        e = g.off[u + 1];
                    }
                    end += e - s;
                    T.lt_delta[wv * 64 + lane] = s - (end - (e - s));
                    T.lt_end[wv * 64 + lane] = end;
                    T.lt_row[wv * 64 + lane] = row;
                }
                const int64_t total = end;
                for (int64_t pos = 0; pos < total; ++pos) {
                    // the lane's cursor walks the table; a lane's positions ascend, so
                    // finding the list from entry 0 visits the same entries
                    int c = 0;
                    while (pos >= T.lt_end[wv * 64 + c]) ++c;
                    const int64_t q = pos + T.lt_delta[wv * 64 + c];
                    if (q < 0 || q >= g.m) { fprintf(stderr, "LDS replay: list entry %ld outside the graph\n", (long)q); abort(); }
                    const int32_t w = g.idx[q];
                    const int i = T.lt_row[wv * 64 + c];
                    if (!bmode) {
                        const uint32_t h = filter_hash(w);
                        if (!((T.flt[h >> 5] >> (h & 31u)) & 1u)) continue;
                    }
                    const int j = member_find(T, w, first, last, bmode);
                    if (j < 0) continue;
                    if (need == 2) {
                        mine += 1;
                        T.cnt[j] += 1;
                        T.cnt[i] += 1;
                    } else {
                        T.rows[(long)i * T.RS + (j >> 5)] |= 1u << (j & 31);
                        T.rows[(long)j * T.RS + (i >> 5)] |= 1u << (i & 31);
                    }
                }
            }
        }
        // no bit at or above d may be set in rows 0..d-1
        for (int x = 0; x < d; ++x)
            for (int q = 0; q < T.W; ++q) {
                const uint32_t b = T.rows[(long)x * T.RS + q];
                for (int t = 0; t < 32; ++t)
                    if ((b >> t) & 1u && q * 32 + t >= d) { fprintf(stderr, "LDS replay: stray bit\n"); abort(); }
            }
        if (need >= 3) {
            g_item = "pair phase";
            const int pneed = need - 2;
            const bool triples = T.W == 2 && pneed >= 4;
            Ring3 q3;
            const bool dyn = T.TW > 1 && pneed >= 2;
            int next = T.TW;          // team row counter
            for (int wv = 0; wv < T.TW; ++wv) {
                unsigned head = 0, tail = 0;
                int xi = wv, claim = 0;
                if (dyn) claim = next++;
                const int B = T.W / 2;
                while (true) {
                    const int row = xi;
                    if (row >= d) break;
                    unsigned pre[64], cntl[64];
                    uint32_t bitsl[64];
                    unsigned acc = 0;
                    for (int lane = 0; lane < 64; ++lane) {
                        const int gg = lane * B;
                        const long base = (long)row * T.RS + (gg >> 5);
                        const int sh = gg & 31;
                        uint64_t win = T.rows[base];
                        if (sh + B > 32) win |= (uint64_t)T.rows[base + 1] << 32;
                        uint32_t bits = (uint32_t)(win >> sh) & (uint32_t)((1ull << B) - 1);
                        const int lim = row - gg;
                        bits &= lim >= B ? ~0u : (lim <= 0 ? 0u : ((1u << lim) - 1u));
                        bitsl[lane] = bits;
                        cntl[lane] = (unsigned)popc(bits);
                        acc += cntl[lane];
                        pre[lane] = acc;
                    }
                    const unsigned end = tail + acc;
                    for (int lane = 0; lane < 64; ++lane) {
                        unsigned pos = tail + pre[lane] - cntl[lane];
                        uint32_t bits = bitsl[lane];
                        while (bits) {
                            const int b = __builtin_ctz(bits);
                            bits &= bits - 1;
                            T.ring[(long)wv * T.RING + (pos & (T.RING - 1))] = ((uint32_t)row << 16) | (uint32_t)(lane * B + b);
                            ++pos;
                        }
                    }
                    if (end - head > (unsigned)T.RING) { fprintf(stderr, "LDS replay: ring overrun\n"); abort(); }
                    while (end - head >= 64) {
                        if (triples) {
                            uint32_t pp[64];
                            for (int lane = 0; lane < 64; ++lane) pp[lane] = T.ring[(long)wv * T.RING + ((head + lane) & (T.RING - 1))];
                            mine += deal3(T, d, q3, pp, 64, pneed);
                        } else {
                            for (int lane = 0; lane < 64; ++lane) {
                                const uint32_t p = T.ring[(long)wv * T.RING + ((head + lane) & (T.RING - 1))];
                                mine += do_pair(T, d, (int)(p & 0xffffu), (int)(p >> 16), pneed);
                            }
                        }
                        head += 64;
                    }
                    tail = end;
                    if (dyn) {
                        xi = claim;
                        if (xi < d) claim = next++;
                    } else {
                        xi += T.TW;
                    }
                }
                if (triples) {
                    uint32_t pp[64];
                    const int nv = (int)(tail - head);
                    for (int lane = 0; lane < 64; ++lane) pp[lane] = T.ring[(long)wv * T.RING + ((head + lane) & (T.RING - 1))];
                    if (nv > 0) mine += deal3(T, d, q3, pp, nv, pneed);
                    for (int lane = 0; lane < (int)(q3.tail - q3.head); ++lane) mine += take3(T, d, q3.r[(q3.head + lane) & 511u], pneed);
                } else {
                    for (int lane = 0; lane < (int)(tail - head); ++lane) {
                        const uint32_t p = T.ring[(long)wv * T.RING + ((head + lane) & (T.RING - 1))];
                        mine += do_pair(T, d, (int)(p & 0xffffu), (int)(p >> 16), pneed);
                    }
                }
            }
        }
    }
    g_item = "flush";
    for (int i = 0; i < d; ++i) pv[T.S[i]] += T.cnt[i];
    pv[root] += mine;
    return mine;
}

}  // namespace

extern "C" uint64_t lds_replay_count(int64_t n, const int64_t *off, const int32_t *idx, int k, int span_max,
                                     uint64_t *pv, int64_t *items_out) {
    Graph g{n, off, idx, off[n]};
    Team tiers[2] = {Team(2), Team(4)};
    uint64_t total = 0;
    int64_t items = 0;
    for (int64_t v = 0; v < n; ++v) pv[v] = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = off[v + 1] - off[v];
        if (d < k - 1) continue;
        if (d > 128) { fprintf(stderr, "LDS replay: models the two smallest tiers only\n"); abort(); }
        total += process_root(tiers[d <= 64 ? 0 : 1], g, k, (int32_t)v, span_max, pv);
        ++items;
    }
    if (items_out) *items_out = items;
    return total;
}
