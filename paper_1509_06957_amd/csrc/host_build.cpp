// Host-side part of index construction: the sparse projection vectors
// (paper Sec. II-B, one vector per tree level per Sec. II-C) and the trees of
// Alg. 1-2 with median splits (Sec. II-A).
//
// The projection vectors are drawn on the host so that every build of the
// same (seed, tree, level, feature) gives the same float32 values; they are
// tiny (T*depth*d draws).  Trees are grown one per host thread.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "mrpt_internal.h"

namespace mrpt {

namespace {

// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): per round two
// 64x64 -> 128-bit products of counter words 0 and 2 with fixed multipliers;
// the high halves are mixed with the remaining counter words and the key, and
// the key advances by two Weyl increments between rounds.
struct Philox4x64 {
    static constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL;
    static constexpr uint64_t kMulB = 0xCA5A826395121157ULL;
    static constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ULL;
    static constexpr uint64_t kWeylB = 0xBB67AE8584CAA73BULL;

    static void block(uint64_t x[4], uint64_t ka, uint64_t kb) {
        for (int round = 0; round < 10; ++round) {
            const unsigned __int128 pa = (unsigned __int128)kMulA * x[0];
            const unsigned __int128 pb = (unsigned __int128)kMulB * x[2];
            const uint64_t y0 = (uint64_t)(pb >> 64) ^ x[1] ^ ka;
            const uint64_t y1 = (uint64_t)pb;
            const uint64_t y2 = (uint64_t)(pa >> 64) ^ x[3] ^ kb;
            const uint64_t y3 = (uint64_t)pa;
            x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
            ka += kWeylA;
            kb += kWeylB;
        }
    }
};

// The entry for (tree t, level lv, feature i) is a pure function of these
// four numbers and the seed: counter (i, lv, t, 0), key (seed, 0).  Word 0
// gives a 53-bit uniform that selects the entry (Bernoulli(a), or by rank in
// the exact-count mode); words 1 and 2 give the two uniforms of a Box-Muller
// standard normal evaluated in double.
struct EntryDraw {
    double select;   // [0, 1)
    float normal;
};

inline EntryDraw draw_entry(uint64_t seed, int32_t t, int32_t lv, int32_t i) {
    uint64_t x[4] = {(uint64_t)i, (uint64_t)lv, (uint64_t)t, 0};
    Philox4x64::block(x, seed, 0);
    constexpr double kInv53 = 1.0 / 9007199254740992.0;  // 2^-53
    const double u1 = (double)((x[1] >> 11) + 1) * kInv53;  // (0, 1]
    const double u2 = (double)(x[2] >> 11) * kInv53;        // [0, 1)
    const double r = std::sqrt(-2.0 * std::log(u1));
    return {(double)(x[0] >> 11) * kInv53, (float)(r * std::cos(6.283185307179586 * u2))};
}

}  // namespace

int32_t exact_nnz_count(int32_t d, float a) {
    const double m = std::ceil((double)a * (double)d);
    return (int32_t)std::min<double>(std::max(m, 1.0), (double)d);
}

void generate_projection(int32_t d, int32_t T, int32_t depth, float a, uint64_t seed, bool exact,
                         std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                         std::vector<float>& val) {
    const int64_t rows = (int64_t)T * depth;
    rowptr.assign(rows + 1, 0);
    col.clear();
    val.clear();
    const double ad = (double)a;
    const int32_t m = exact_nnz_count(d, a);
    std::vector<EntryDraw> e((size_t)d);
    std::vector<int32_t> pick((size_t)d);
    for (int32_t t = 0; t < T; ++t)
        for (int32_t lv = 0; lv < depth; ++lv) {
            for (int32_t i = 0; i < d; ++i) e[i] = draw_entry(seed, t, lv, i);
            if (exact) {
                // the m features of smallest (select, feature): a uniformly
                // random m-subset (Sec. II-D footnote), then ascending features
                for (int32_t i = 0; i < d; ++i) pick[i] = i;
                std::nth_element(pick.begin(), pick.begin() + (m - 1), pick.end(), [&](int32_t x, int32_t y) {
                    return e[x].select < e[y].select || (e[x].select == e[y].select && x < y);
                });
                std::sort(pick.begin(), pick.begin() + m);
                for (int32_t j = 0; j < m; ++j) {
                    const int32_t i = pick[j];
                    if (e[i].normal != 0.0f) {
                        col.push_back(i);
                        val.push_back(e[i].normal);
                    }
                }
            } else {
                for (int32_t i = 0; i < d; ++i) {
                    if (e[i].select < ad && e[i].normal != 0.0f) {
                        col.push_back(i);
                        val.push_back(e[i].normal);
                    }
                }
            }
            rowptr[(int64_t)t * depth + lv + 1] = (int32_t)col.size();
        }
}

// Leaf sizes depend only on (n, depth): a node with m points keeps
// ceil(m/2) on the left.  Computed level by level from the root.
void leaf_offsets(int64_t n, int32_t depth, std::vector<int64_t>& off) {
    std::vector<int64_t> sizes(1, n), next;
    for (int32_t lv = 0; lv < depth; ++lv) {
        next.resize(sizes.size() * 2);
        for (size_t j = 0; j < sizes.size(); ++j) {
            next[2 * j] = (sizes[j] + 1) / 2;
            next[2 * j + 1] = sizes[j] / 2;
        }
        sizes.swap(next);
    }
    off.assign(sizes.size() + 1, 0);
    for (size_t j = 0; j < sizes.size(); ++j) off[j + 1] = off[j] + sizes[j];
}

namespace {

struct Key {
    float p;
    int32_t id;
};
inline bool key_less(const Key& x, const Key& y) {
    return x.p < y.p || (x.p == y.p && x.id < y.id);
}

// One tree: projections of every point onto its depth vectors (float32,
// fused multiply-add in ascending feature order from +0), then level by
// level each node is cut by rank: its ceil(m/2) smallest (projection, id)
// keys go left.  The split stored for queries is the largest left value for
// odd m and the float32 midpoint of the two middle values for even m.
void grow_one(const float* X, int64_t n, int32_t d, int32_t depth, const int32_t* rp,
              const int32_t* cl, const float* vl, const std::vector<std::vector<int64_t>>& level_off,
              float* splits, int32_t* perm) {
    std::vector<float> P((size_t)n * (size_t)std::max(depth, 1));  // level-major: P[lv*n + x]
    for (int32_t lv = 0; lv < depth; ++lv) {
        const int32_t b = rp[lv], e = rp[lv + 1];
        float* Pl = P.data() + (size_t)lv * n;
        for (int64_t x = 0; x < n; ++x) {
            const float* xr = X + x * d;
            float acc = 0.0f;
            for (int32_t j = b; j < e; ++j) acc = std::fmaf(xr[cl[j]], vl[j], acc);
            Pl[x] = acc == 0.0f ? 0.0f : acc;
        }
    }
    std::vector<int32_t> ids((size_t)n);
    for (int64_t i = 0; i < n; ++i) ids[i] = (int32_t)i;
    std::vector<Key> keys;
    for (int32_t lv = 0; lv < depth; ++lv) {
        const std::vector<int64_t>& lo = level_off[lv];  // node boundaries at this level
        const float* Pl = P.data() + (size_t)lv * n;
        const int64_t first_node = ((int64_t)1 << lv) - 1;
        for (size_t j = 0; j + 1 < lo.size(); ++j) {
            const int64_t b = lo[j], m = lo[j + 1] - lo[j];
            keys.resize((size_t)m);
            for (int64_t i = 0; i < m; ++i) keys[i] = Key{Pl[ids[b + i]], ids[b + i]};
            const int64_t nl = (m + 1) / 2;
            std::nth_element(keys.begin(), keys.begin() + (nl - 1), keys.end(), key_less);
            const float left_max = keys[nl - 1].p;
            float split = left_max;
            if ((m & 1) == 0) {
                float right_min = keys[nl].p;
                for (int64_t i = nl + 1; i < m; ++i) right_min = std::min(right_min, keys[i].p);
                const float sum = left_max + right_min;
                split = sum * 0.5f;
            }
            splits[first_node + (int64_t)j] = split;
            for (int64_t i = 0; i < m; ++i) ids[b + i] = keys[i].id;
        }
    }
    const std::vector<int64_t>& leaves = level_off[depth];
    for (size_t L = 0; L + 1 < leaves.size(); ++L)
        std::sort(ids.begin() + leaves[L], ids.begin() + leaves[L + 1]);
    std::memcpy(perm, ids.data(), sizeof(int32_t) * (size_t)n);
}

}  // namespace

void grow_trees_host(const float* X, int64_t n, int32_t d, int32_t T, int32_t depth,
                     const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                     const std::vector<float>& val, HostTrees& out) {
    const int64_t nsplit = ((int64_t)1 << depth) - 1;
    out.splits.assign((size_t)T * (size_t)nsplit, 0.0f);
    out.perm.assign((size_t)T * (size_t)n, 0);
    // node boundaries per level (level depth = the leaves)
    std::vector<std::vector<int64_t>> level_off((size_t)depth + 1);
    for (int32_t lv = 0; lv <= depth; ++lv) leaf_offsets(n, lv, level_off[lv]);
    out.off = level_off[depth];

    unsigned hw = std::thread::hardware_concurrency();
    int nth = (int)std::max(1u, std::min(hw == 0 ? 1u : hw, 16u));
    nth = std::min(nth, T);
    std::vector<std::thread> pool;
    for (int w = 0; w < nth; ++w)
        pool.emplace_back([&, w]() {
            for (int32_t t = w; t < T; t += nth) {
                std::vector<int32_t> rp((size_t)depth + 1);
                const int64_t r0 = (int64_t)t * depth;
                for (int32_t lv = 0; lv <= depth; ++lv) rp[lv] = rowptr[r0 + lv];
                grow_one(X, n, d, depth, rp.data(), col.data(), val.data(), level_off,
                         out.splits.data() + (size_t)t * nsplit, out.perm.data() + (size_t)t * n);
            }
        });
    for (auto& th : pool) th.join();
}

}  // namespace mrpt
