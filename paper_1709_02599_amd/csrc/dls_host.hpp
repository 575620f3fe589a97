// dls_host.hpp -- host-side planning for the DLS counting library: the cell
// fill order (Sec. 2.3), workunit splitting (Sec. 5.2), and hourglass
// symmetry breaking (Sec. 4.2-4.3, Alg. 5-6).  No GPU code here.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace dls {

constexpr int kMaxN = 16;
constexpr uint8_t kEmpty = 0xFF;

// Fill order of the empty cells.  `assigned` has n*n entries (nonzero =
// assigned); `first` (may be empty) lists cells that must come before all
// others.  With vs, only left-half cells are listed and each pick also
// assigns its mirror (i, n-1-j).  `variant` 0 is the rule of Sec. 2.3; the
// others change weights or tie-breaks for the autotuner (the count never
// depends on the order): 1 column-major ties, 2 rows weigh double, 3 columns
// weigh double, 4 no forced-cell rule, 5 last cell on ties, 6 diagonals
// weigh double, 7 diagonals ignored.
constexpr int kOrderVariants = 8;
std::vector<int> fill_order(int n, bool vs, const uint8_t *assigned,
                            const std::vector<int> &first, int variant = 0);

// Hourglass cells (Sec. 4.2): rows 0 and n-1 and both diagonals, row-major.
std::vector<int> hourglass_cells(int n);

// Bitmask occupancy of a partial square (the Rows/Columns/MD/AD words of
// Sec. 3).  place() checks and marks one cell; unplace() undoes it.
struct Board {
    int n = 0;
    uint32_t rows[kMaxN] = {0}, cols[kMaxN] = {0}, md = 0, ad = 0;
    uint8_t cell[kMaxN * kMaxN];

    void reset(int n_);
    bool can(int i, int j, int v) const;
    void place(int i, int j, int v);
    void unplace(int i, int j, int v);
    // VS: place v at (i,j) and n-1-v at its mirror; false if impossible.
    bool can_pair(int i, int j, int v) const;
    void place_pair(int i, int j, int v);
    void unplace_pair(int i, int j, int v);
    // Load a prefix; false if its assigned cells break a constraint.
    bool load(const uint8_t *sq, bool vs);
};

// Complete a VS prefix by mirror pairs; false if a pair is inconsistent.
bool vs_complete(int n, const uint8_t *in, uint8_t *out);

// Canonicity of an hourglass design (Alg. 5) through the transformation
// group built as the product of the three tables of Alg. 5.
class HourglassGroup {
  public:
    explicit HourglassGroup(int n);
    int size() const { return (int)p_.size(); }
    // 0 if some image is lexicographically smaller, else the class power.
    uint32_t canon(const uint8_t *h) const;
    // image of h under element g (renormalised by row 0), for tests.
    void apply(int g, const uint8_t *h, uint8_t *out) const;
    // the group as a table [size()][cells().size()]: entry (g, k) is the
    // index (into cells()) of the hourglass cell whose value lands on
    // hourglass cell k under g
    std::vector<uint8_t> src_table() const;
    const std::vector<int> &cells() const { return hc_; }

  private:
    int n_;
    std::vector<int> hc_;                        // hourglass cells, row-major
    std::vector<std::vector<int8_t>> p_, q_;     // T[i][j] = H[p[i]][q[j]]
    std::vector<std::vector<int>> src_;          // per g: source cell of hc_[k]
};

// Depth-first enumeration of consistent assignments of `cells` (in order)
// on top of `base`.  emit(square, mult) is called for each leaf; with a
// group, leaves at hourglass level `hg_level` are canonicalised and only
// canonical designs are extended (mult = class power).  Returns the number of
// emitted prefixes.  Multithreaded over the subtrees at a shallow level when
// threads > 1 (emit is then called from several threads, in an order that is
// made deterministic by the caller's sort).
struct SplitSpec {
    int n = 0;
    bool vs = false;
    std::vector<int> cells;              // cells to assign, in order
    const HourglassGroup *group = nullptr;
    int hg_level = -1;                   // #cells after which the hourglass is complete
};

int64_t split_count(const SplitSpec &spec, const uint8_t *base);
// Writes prefixes (and mult) in deterministic depth-first order.
int64_t split_write(const SplitSpec &spec, const uint8_t *base, uint8_t *out, uint32_t *mult,
                    int64_t cap);
// Visit prefixes at the given increasing positions.
int64_t split_select(const SplitSpec &spec, const uint8_t *base, const int64_t *idx, int64_t k,
                     uint8_t *out);

int host_threads();

// Cost of a fill order: the number of downward DFS steps (entries into
// levels below the first) that the search kernels take over the given
// prefixes when they fill `order` (with vs: left-half cells) in that order,
// and the number of squares reached.  -1 if an order cell is assigned in a
// prefix.  Multithreaded over prefixes.
int order_cost(int n, bool vs, const std::vector<int> &order, const uint8_t *prefixes, int64_t num,
               uint64_t *steps_out, uint64_t *leaves_out);

}  // namespace dls
