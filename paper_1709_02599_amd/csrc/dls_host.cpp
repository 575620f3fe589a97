// dls_host.cpp -- fill order (Sec. 2.3), workunit split (Sec. 5.2) and
// hourglass symmetry breaking (Sec. 4.2-4.3, Alg. 5-6) on the host.
#include "dls_host.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <numeric>
#include <thread>

namespace dls {

int host_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 1;
    if (t > 64) t = 64;
    return (int)t;
}

// ---------------------------------------------------------------------------
// fill order (Sec. 2.3)
// ---------------------------------------------------------------------------

std::vector<int> fill_order(int n, bool vs, const uint8_t *assigned, const std::vector<int> &first,
                            int variant) {
    const int wr = variant == 2 ? 2 : 1, wc = variant == 3 ? 2 : 1;
    const int wd = variant == 6 ? 2 : (variant == 7 ? 0 : 1);
    const bool forced_rule = variant != 4;
    const int nn = n * n;
    std::vector<uint8_t> a(nn, 0), pri(nn, 0);
    for (int c = 0; c < nn; ++c) a[c] = assigned[c] ? 1 : 0;
    auto mirror = [n](int c) { return (c / n) * n + (n - 1 - c % n); };
    auto is_left = [n](int c) { return 2 * (c % n) <= n - 1; };
    auto rep = [&](int c) { return (!vs || is_left(c)) ? c : mirror(c); };
    for (int c : first)
        if (c >= 0 && c < nn) pri[rep(c)] = 1;

    std::vector<int> order;
    for (;;) {
        // counts of assigned cells per line
        int r[kMaxN] = {0}, col[kMaxN] = {0}, md = 0, ad = 0;
        for (int c = 0; c < nn; ++c) {
            if (!a[c]) continue;
            int i = c / n, j = c % n;
            r[i]++;
            col[j]++;
            if (i == j) md++;
            if (i + j == n - 1) ad++;
        }
        std::vector<uint8_t> allowed(nn, 0);
        bool any = false, any_pri = false;
        for (int c = 0; c < nn; ++c) {
            if (a[c] || (vs && !is_left(c))) continue;
            allowed[c] = 1;
            any = true;
            if (pri[c]) any_pri = true;
        }
        if (!any) break;
        if (any_pri)
            for (int c = 0; c < nn; ++c)
                if (!pri[c]) allowed[c] = 0;

        // forced rule: a line with exactly n-1 assigned cells
        int pick = -1;
        auto consider_forced = [&](int c) {
            c = rep(c);
            if (forced_rule && allowed[c] && (pick < 0 || c < pick)) pick = c;
        };
        for (int i = 0; i < n; ++i)
            if (r[i] == n - 1)
                for (int j = 0; j < n; ++j)
                    if (!a[i * n + j]) consider_forced(i * n + j);
        for (int j = 0; j < n; ++j)
            if (col[j] == n - 1)
                for (int i = 0; i < n; ++i)
                    if (!a[i * n + j]) consider_forced(i * n + j);
        if (md == n - 1)
            for (int i = 0; i < n; ++i)
                if (!a[i * n + i]) consider_forced(i * n + i);
        if (ad == n - 1)
            for (int i = 0; i < n; ++i)
                if (!a[i * n + n - 1 - i]) consider_forced(i * n + n - 1 - i);

        if (pick < 0) {  // most constrained cell, first in row-major order on ties
            int best = -1;
            for (int t = 0; t < nn; ++t) {
                // scan order: row-major (paper), column-major, or reversed
                const int c = variant == 1 ? (t % n) * n + t / n : (variant == 5 ? nn - 1 - t : t);
                if (!allowed[c]) continue;
                int i = c / n, j = c % n;
                int v = wr * r[i] + wc * col[j] + wd * ((i == j ? md : 0) + (i + j == n - 1 ? ad : 0));
                if (v > best) {
                    best = v;
                    pick = c;
                }
            }
        }
        a[pick] = 1;
        if (vs) a[mirror(pick)] = 1;
        order.push_back(pick);
    }
    return order;
}

std::vector<int> hourglass_cells(int n) {
    std::vector<int> cells;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i == 0 || i == n - 1 || i == j || i + j == n - 1) cells.push_back(i * n + j);
    return cells;
}

// ---------------------------------------------------------------------------
// bitmask board
// ---------------------------------------------------------------------------

void Board::reset(int n_) {
    n = n_;
    std::memset(rows, 0, sizeof(rows));
    std::memset(cols, 0, sizeof(cols));
    md = ad = 0;
    std::memset(cell, kEmpty, sizeof(cell));
}

bool Board::can(int i, int j, int v) const {
    uint32_t b = 1u << v;
    uint32_t cr = rows[i] | cols[j];
    if (i == j) cr |= md;
    if (i + j == n - 1) cr |= ad;
    return (cr & b) == 0;
}

void Board::place(int i, int j, int v) {
    uint32_t b = 1u << v;
    rows[i] |= b;
    cols[j] |= b;
    if (i == j) md |= b;
    if (i + j == n - 1) ad |= b;
    cell[i * n + j] = (uint8_t)v;
}

void Board::unplace(int i, int j, int v) {
    uint32_t b = 1u << v;
    rows[i] &= ~b;
    cols[j] &= ~b;
    if (i == j) md &= ~b;
    if (i + j == n - 1) ad &= ~b;
    cell[i * n + j] = kEmpty;
}

bool Board::can_pair(int i, int j, int v) const {
    int jj = n - 1 - j, w = n - 1 - v;
    if (jj == j) return v == w && can(i, j, v);
    if (!can(i, j, v)) return false;
    Board t = *this;
    t.place(i, j, v);
    return t.can(i, jj, w);
}

void Board::place_pair(int i, int j, int v) {
    place(i, j, v);
    if (n - 1 - j != j) place(i, n - 1 - j, n - 1 - v);
}

void Board::unplace_pair(int i, int j, int v) {
    if (n - 1 - j != j) unplace(i, n - 1 - j, n - 1 - v);
    unplace(i, j, v);
}

bool Board::load(const uint8_t *sq, bool vs) {
    (void)vs;
    for (int c = 0; c < n * n; ++c) {
        int v = sq[c];
        if (v == kEmpty) continue;
        int i = c / n, j = c % n;
        if (!can(i, j, v)) return false;
        place(i, j, v);
    }
    return true;
}

bool vs_complete(int n, const uint8_t *in, uint8_t *out) {
    std::memcpy(out, in, (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            int c = i * n + j, m = i * n + (n - 1 - j);
            if (in[c] == kEmpty) continue;
            int w = n - 1 - in[c];
            if (out[m] == kEmpty)
                out[m] = (uint8_t)w;
            else if (out[m] != w)
                return false;
        }
    return true;
}

// ---------------------------------------------------------------------------
// hourglass transformation group: the three tables of Alg. 5
// ---------------------------------------------------------------------------

HourglassGroup::HourglassGroup(int n) : n_(n) {
    hc_ = hourglass_cells(n);
    const int m = n / 2;
    std::vector<int8_t> id(n);
    std::iota(id.begin(), id.end(), 0);
    // TR_0: identity and the vertical mirror (columns reversed)
    std::vector<std::vector<int8_t>> tr0_q(2, id);
    for (int j = 0; j < n; ++j) tr0_q[1][j] = (int8_t)(n - 1 - j);
    // TR_1: every subset of the symmetric pairs {k, n-1-k} swapped, rows and columns together
    std::vector<std::vector<int8_t>> tr1;
    for (int s = 0; s < (1 << m); ++s) {
        std::vector<int8_t> p = id;
        for (int k = 0; k < m; ++k)
            if (s >> k & 1) std::swap(p[k], p[n - 1 - k]);
        tr1.push_back(p);
    }
    // TR_2: every permutation of the pairs 1..m-1 (pair 0 = rows 0 and n-1 stays)
    std::vector<std::vector<int8_t>> tr2;
    std::vector<int> perm;
    for (int k = 1; k < m; ++k) perm.push_back(k);
    do {
        std::vector<int8_t> p = id;
        for (int t = 0; t < (int)perm.size(); ++t) {
            int k = t + 1, to = perm[t];
            p[k] = (int8_t)to;
            p[n - 1 - k] = (int8_t)(n - 1 - to);
        }
        tr2.push_back(p);
    } while (std::next_permutation(perm.begin(), perm.end()));
    // products: p = tr1 o tr2 on rows, q = tr0 o p on columns
    for (auto &q0 : tr0_q)
        for (auto &p1 : tr1)
            for (auto &p2 : tr2) {
                std::vector<int8_t> p(n), q(n);
                for (int x = 0; x < n; ++x) p[x] = p1[p2[x]];
                for (int x = 0; x < n; ++x) q[x] = p[q0[x]];
                p_.push_back(p);
                q_.push_back(q);
            }
    for (size_t g = 0; g < p_.size(); ++g) {
        std::vector<int> src(hc_.size());
        for (size_t k = 0; k < hc_.size(); ++k) {
            int i = hc_[k] / n, j = hc_[k] % n;
            src[k] = p_[g][i] * n + q_[g][j];
        }
        src_.push_back(src);
    }
}

std::vector<uint8_t> HourglassGroup::src_table() const {
    std::vector<int> pos((size_t)n_ * n_, -1);
    for (size_t k = 0; k < hc_.size(); ++k) pos[hc_[k]] = (int)k;
    std::vector<uint8_t> t;
    t.reserve(src_.size() * hc_.size());
    for (const auto &src : src_)
        for (int c : src) t.push_back((uint8_t)pos[c]);
    return t;
}

uint32_t HourglassGroup::canon(const uint8_t *h) const {
    const int n = n_;
    int stab = 0;
    uint8_t rename[kMaxN];
    for (size_t g = 0; g < src_.size(); ++g) {
        const int *src = src_[g].data();
        // image row 0 is hc_[0..n-1]; renaming makes it 0..n-1
        for (int j = 0; j < n; ++j) rename[h[src[j]]] = (uint8_t)j;
        int cmp = 0;
        for (size_t k = n; k < hc_.size(); ++k) {
            uint8_t img = rename[h[src[k]]], own = h[hc_[k]];
            if (img != own) {
                cmp = img < own ? -1 : 1;
                break;
            }
        }
        if (cmp < 0) return 0;
        if (cmp == 0) ++stab;
    }
    // class power = |G| / |stabiliser| (orbit-stabiliser)
    return (uint32_t)(src_.size() / (size_t)stab);
}

void HourglassGroup::apply(int g, const uint8_t *h, uint8_t *out) const {
    const int n = n_;
    uint8_t rename[kMaxN];
    const int *src = src_[g].data();
    for (int j = 0; j < n; ++j) rename[h[src[j]]] = (uint8_t)j;
    std::memset(out, kEmpty, (size_t)n * n);
    for (size_t k = 0; k < hc_.size(); ++k) out[hc_[k]] = rename[h[src[k]]];
}

// ---------------------------------------------------------------------------
// split (workunits of Sec. 5.2), optionally through canonical hourglasses
// ---------------------------------------------------------------------------

namespace {

struct Walker {
    const SplitSpec *s;
    Board b;
    uint32_t mult = 1;
    int stop = 0;

    template <class F>
    void dfs(int lvl, F &leaf) {
        if (s->group && lvl == s->hg_level) {
            mult = s->group->canon(b.cell);
            if (!mult) return;
        }
        if (lvl == stop) {
            leaf(*this);
            return;
        }
        const int n = s->n, c = s->cells[lvl], i = c / n, j = c % n;
        for (int v = 0; v < n; ++v) {
            if (s->vs) {
                if (!b.can_pair(i, j, v)) continue;
                b.place_pair(i, j, v);
                dfs(lvl + 1, leaf);
                b.unplace_pair(i, j, v);
            } else {
                if (!b.can(i, j, v)) continue;
                b.place(i, j, v);
                dfs(lvl + 1, leaf);
                b.unplace(i, j, v);
            }
        }
    }
};

bool init_board(const SplitSpec &s, const uint8_t *base, Board &b) {
    b.reset(s.n);
    return b.load(base, s.vs);
}

// seeds: the prefixes at a shallow level L0, enough to spread over threads
int choose_seed_level(const SplitSpec &s, const uint8_t *base, std::vector<uint8_t> &seeds,
                      std::vector<uint32_t> &seed_mult) {
    const int nn = s.n * s.n;
    const int total = (int)s.cells.size();
    const int want = 64 * host_threads();
    int level = 0;
    seeds.assign(base, base + nn);
    seed_mult.assign(1, 1);
    while (level < total && (int64_t)seed_mult.size() < want) {
        // never expand across the hourglass level in the seed phase without
        // canonicalising: Walker handles canon at hg_level when it is reached
        Walker w;
        w.s = &s;
        std::vector<uint8_t> next;
        std::vector<uint32_t> next_mult;
        for (size_t k = 0; k < seed_mult.size(); ++k) {
            if (!init_board(s, seeds.data() + k * nn, w.b)) continue;
            w.mult = seed_mult[k];
            w.stop = level + 1;
            auto leaf = [&](Walker &ww) {
                next.insert(next.end(), ww.b.cell, ww.b.cell + nn);
                next_mult.push_back(ww.mult);
            };
            // dfs from `level` assigns exactly one cell (stop = level + 1)
            w.dfs(level, leaf);
        }
        seeds.swap(next);
        seed_mult.swap(next_mult);
        ++level;
        if (seed_mult.empty()) break;
    }
    return level;
}

template <class PerSeed>
void run_seeds(const SplitSpec &s, int level, const std::vector<uint8_t> &seeds,
               const std::vector<uint32_t> &seed_mult, PerSeed per_seed) {
    const int nn = s.n * s.n;
    const int64_t ns = (int64_t)seed_mult.size();
    std::atomic<int64_t> next(0);
    auto worker = [&]() {
        Walker w;
        w.s = &s;
        w.stop = (int)s.cells.size();
        for (;;) {
            int64_t k = next.fetch_add(1);
            if (k >= ns) break;
            if (!init_board(s, seeds.data() + k * nn, w.b)) continue;
            w.mult = seed_mult[k];
            per_seed(k, w, level);
        }
    };
    int nt = std::min<int64_t>(host_threads(), std::max<int64_t>(1, ns));
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

}  // namespace

int64_t split_count(const SplitSpec &s, const uint8_t *base) {
    std::vector<uint8_t> seeds;
    std::vector<uint32_t> sm;
    int level = choose_seed_level(s, base, seeds, sm);
    std::vector<int64_t> per(sm.size(), 0);
    run_seeds(s, level, seeds, sm, [&](int64_t k, Walker &w, int lvl) {
        int64_t c = 0;
        auto leaf = [&](Walker &) { ++c; };
        w.dfs(lvl, leaf);
        per[k] = c;
    });
    return std::accumulate(per.begin(), per.end(), (int64_t)0);
}

int64_t split_write(const SplitSpec &s, const uint8_t *base, uint8_t *out, uint32_t *mult,
                    int64_t cap) {
    const int nn = s.n * s.n;
    std::vector<uint8_t> seeds;
    std::vector<uint32_t> sm;
    int level = choose_seed_level(s, base, seeds, sm);
    std::vector<std::vector<uint8_t>> cells(sm.size());
    std::vector<std::vector<uint32_t>> mults(sm.size());
    run_seeds(s, level, seeds, sm, [&](int64_t k, Walker &w, int lvl) {
        auto &cv = cells[k];
        auto &mv = mults[k];
        auto leaf = [&](Walker &ww) {
            cv.insert(cv.end(), ww.b.cell, ww.b.cell + nn);
            mv.push_back(ww.mult);
        };
        w.dfs(lvl, leaf);
    });
    int64_t total = 0;
    for (auto &m : mults) total += (int64_t)m.size();
    if (out == nullptr || total > cap) return total;
    int64_t pos = 0;
    for (size_t k = 0; k < mults.size(); ++k) {
        std::memcpy(out + pos * nn, cells[k].data(), cells[k].size());
        if (mult) std::memcpy(mult + pos, mults[k].data(), mults[k].size() * sizeof(uint32_t));
        pos += (int64_t)mults[k].size();
    }
    return total;
}

int64_t split_select(const SplitSpec &s, const uint8_t *base, const int64_t *idx, int64_t k,
                     uint8_t *out) {
    const int nn = s.n * s.n;
    std::vector<uint8_t> seeds;
    std::vector<uint32_t> sm;
    int level = choose_seed_level(s, base, seeds, sm);
    const int64_t ns = (int64_t)sm.size();
    // pass 1: size of every seed's subtree
    std::vector<int64_t> sz(ns, 0);
    run_seeds(s, level, seeds, sm, [&](int64_t q, Walker &w, int lvl) {
        int64_t c = 0;
        auto leaf = [&](Walker &) { ++c; };
        w.dfs(lvl, leaf);
        sz[q] = c;
    });
    std::vector<int64_t> off(ns + 1, 0);
    for (int64_t q = 0; q < ns; ++q) off[q + 1] = off[q] + sz[q];
    const int64_t total = off[ns];
    if (k > 0 && idx[k - 1] >= total) return -total - 1;
    // pass 2: visit only the seeds that hold requested positions
    std::vector<int64_t> first(ns, -1), last(ns, -1);
    for (int64_t t = 0, q = 0; t < k; ++t) {
        while (off[q + 1] <= idx[t]) ++q;
        if (first[q] < 0) first[q] = t;
        last[q] = t;
    }
    run_seeds(s, level, seeds, sm, [&](int64_t q, Walker &w, int lvl) {
        if (first[q] < 0) return;
        int64_t pos = off[q], t = first[q];
        auto leaf = [&](Walker &ww) {
            if (t <= last[q] && pos == idx[t]) {
                std::memcpy(out + t * nn, ww.b.cell, nn);
                ++t;
            }
            ++pos;
        };
        w.dfs(lvl, leaf);
    });
    return total;
}

}  // namespace dls

// ---------------------------------------------------------------------------
// cost of a fill order: the DFS steps the search kernels would take
// ---------------------------------------------------------------------------

namespace dls {

namespace {

struct CostLevel {
    int i, j;
    uint32_t md, ad;  // all-ones if the cell lies on the diagonal
};

struct CostState {
    int n;
    bool vs;
    uint32_t rows[kMaxN], cols[kMaxN], md, ad;
};

// Entries into levels 1..last below level `lvl` (each entry is one downward
// step of the kernels' search); leaves counted at the last level.
void cost_dfs(CostState &s, const std::vector<CostLevel> &lv, int lvl, uint64_t &steps, uint64_t &leaves) {
    const CostLevel &c = lv[lvl];
    const uint32_t all = (1u << s.n) - 1u;
    const uint32_t cand = all & ~(s.rows[c.i] | s.cols[c.j] | (s.md & c.md) | (s.ad & c.ad));
    if (lvl + 1 == (int)lv.size()) {
        leaves += (uint64_t)__builtin_popcount(cand);
        return;
    }
    for (uint32_t l = cand; l; l &= l - 1u) {
        const uint32_t b = l & (0u - l);
        const int v = __builtin_ctz(b);
        const uint32_t rb = s.vs ? (1u << (s.n - 1 - v)) : 0u;
        s.rows[c.i] ^= b | rb;
        s.cols[c.j] ^= b;
        const uint32_t dm = (b & c.md) | (rb & c.ad), da = (b & c.ad) | (rb & c.md);
        s.md ^= dm;
        s.ad ^= da;
        ++steps;
        cost_dfs(s, lv, lvl + 1, steps, leaves);
        s.rows[c.i] ^= b | rb;
        s.cols[c.j] ^= b;
        s.md ^= dm;
        s.ad ^= da;
    }
}

}  // namespace

int order_cost(int n, bool vs, const std::vector<int> &order, const uint8_t *prefixes, int64_t num,
               uint64_t *steps_out, uint64_t *leaves_out) {
    const int nn = n * n;
    std::vector<CostLevel> lv;
    for (int c : order) {
        const int i = c / n, j = c % n;
        lv.push_back({i, j, i == j ? ~0u : 0u, i + j == n - 1 ? ~0u : 0u});
    }
    std::atomic<int64_t> next(0);
    std::atomic<uint64_t> steps(0), leaves(0);
    std::atomic<int> bad(0);
    auto work = [&]() {
        uint64_t st = 0, le = 0;
        for (;;) {
            const int64_t k = next.fetch_add(1);
            if (k >= num) break;
            const uint8_t *p = prefixes + k * nn;
            std::vector<uint8_t> full(p, p + nn);
            if (vs && !vs_complete(n, p, full.data())) continue;
            Board b;
            b.reset(n);
            if (!b.load(full.data(), vs)) continue;  // inconsistent prefix: no work
            for (int c : order)
                if (b.cell[c] != kEmpty) bad = 1;
            if (lv.empty()) {
                ++le;
                continue;
            }
            CostState s;
            s.n = n;
            s.vs = vs;
            for (int t = 0; t < n; ++t) {
                s.rows[t] = b.rows[t];
                s.cols[t] = b.cols[t];
            }
            s.md = b.md;
            s.ad = b.ad;
            cost_dfs(s, lv, 0, st, le);
        }
        steps += st;
        leaves += le;
    };
    const int th = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, num));
    std::vector<std::thread> pool;
    for (int t = 1; t < th; ++t) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    if (bad) return -1;
    *steps_out = steps;
    *leaves_out = leaves;
    return 0;
}

}  // namespace dls
