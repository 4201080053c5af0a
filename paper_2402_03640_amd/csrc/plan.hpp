// Host-side instance plan: canonical clauses and the two sparse layouts of W
// (clause-major for the scores, variable-major for the adjoint) in the tiled
// column-major form the kernels read.  No HIP in here.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace hms {

// Host buffers of the plan build.  Blocks of 2 MiB or more are mapped apart
// with transparent huge pages requested: the build is bound by the first-touch
// page faults of its fresh buffers, and a 2 MiB page faults once where 4 KiB
// pages fault 512 times.  Smaller blocks come from operator new.
void* build_alloc(std::size_t bytes);
void build_free(void* p, std::size_t bytes) noexcept;

template <class T>
struct BuildAlloc {
    using value_type = T;
    BuildAlloc() = default;
    template <class U>
    BuildAlloc(const BuildAlloc<U>&) {}
    T* allocate(std::size_t n) { return static_cast<T*>(build_alloc(n * sizeof(T))); }
    void deallocate(T* p, std::size_t n) noexcept { build_free(p, n * sizeof(T)); }
    template <class U>
    bool operator==(const BuildAlloc<U>&) const { return true; }
    template <class U>
    bool operator!=(const BuildAlloc<U>&) const { return false; }
};
template <class T>
using PVec = std::vector<T, BuildAlloc<T>>;

constexpr int kTile = 64;          // rows per tile; one wavefront lane per row at R = 1
constexpr int kSeg = 64;           // entries per segment of a split variable row; rows up to kSeg stay whole
constexpr int kSplitDense = 256;   // longest row kept whole when most rows exceed kSeg
constexpr int kWideSegs = 1024;    // variables with more segments combine over 1024 slots (else 64)
constexpr uint32_t kSign = 0x80000000u;
constexpr uint32_t kIdx = 0x7fffffffu;
constexpr uint32_t kNoSlot = 0xffffffffu;  // clause-side entry with no occurrence (padding)

// Per-tile descriptor (16 bytes).  Entry (c, rowin) of the tile sits at
// ent[base + c * kTile + rowin]; rows rowin >= nreal are padding.
struct TileDesc {
    uint32_t base;   // first entry of the tile
    uint32_t len;    // entries per row (the tile's longest row; shorter rows are padded)
    uint32_t nreal;  // real rows in the tile
    uint32_t flags;  // clause side: 1 = rows hold a complementary pair (always satisfied)
};

struct HostPlan {
    int32_t n = 0;              // variables as declared
    int32_t m = 0;              // clauses as given (the loss divides by this)
    int64_t lits_in = 0;        // nonzero literals as given
    int32_t m_empty = 0;        // empty clauses: always unsatisfied, score 0
    int32_t m_taut = 0;         // clauses holding v and not-v: always satisfied
    int32_t m_taut_dropped = 0; // tautologies whose every entry cancelled
    int64_t nnz = 0;            // nonzero entries of W over the kernel rows
    // clause weights (weighted MaxSAT); without weights every clause weighs 1
    bool weighted = false;
    int64_t w_total = 0;        // total weight (m without weights): the cost of "all unsatisfied"
    int64_t w_empty = 0;        // total weight of the empty clauses (always unsatisfied)
    PVec<int64_t> c_w;   // [c_tiles * kTile] weight of each kernel row (0 = padding); empty if unweighted

    // clause side (scores / mask / adjoint)
    int32_t mk = 0;             // kernel clause rows
    int32_t c_tiles = 0;
    PVec<TileDesc> c_tile;
    PVec<uint32_t> c_ent;     // new variable index | sign bit (negated literal)
    PVec<int32_t> c_row_orig; // [c_tiles * kTile] original clause of a row, -1 = padding
    // [c_ent.size()] where each clause-side entry sits on the variable side:
    // the index into v_ent of the same occurrence | its sign bit, or kNoSlot
    // for padding.  Within a tile the map is stored row by row: entry (c, row)
    // of the tile at base + row * len + c (the entries themselves are column
    // by column).  The library builds this map on the device at load; the
    // host copy is filled only by build_slots (the host plan view).
    PVec<uint32_t> c_slot;
    bool slot_ok = false;            // the variable side has fewer than 2^31 entries (slot schedules can run)

    // variable side (transposed sums); rows are whole light variables or
    // fixed-length segments of heavy variables
    int32_t n_act = 0;          // variables with at least one nonzero entry
    int32_t split_len = kSeg;   // longest variable row kept whole
    int32_t n_heavy = 0;        // variables with more than split_len entries
    int32_t seg_rows = 0;       // real segment rows
    int32_t seg_tiles = 0;      // tiles holding segment rows (come first)
    int32_t v_tiles = 0;        // all variable-side tiles
    PVec<TileDesc> v_tile;
    PVec<uint32_t> v_ent;     // clause row index | sign bit
    PVec<int32_t> seg_first;  // [n_heavy + 1] into seg_row
    PVec<int32_t> seg_row;    // segment row of each segment: the identity (rows are in segment order)
    int32_t max_segs = 0;            // most segments of one variable
    int32_t n_heavy_wide = 0;        // heavy variables with more than kWideSegs segments (come first)

    int32_t build_threads = 1;       // host threads the build used (the plan is the same for any count)

    PVec<int32_t> var_old;    // new index -> original (0-based)
    PVec<int32_t> var_new;    // original -> new index
    PVec<int32_t> degree;     // by new index

    int32_t a_rows() const { return c_tiles * kTile + 1; }  // last row stays zero
    int32_t a_zero_row() const { return c_tiles * kTile; }
    int32_t light_row0() const { return seg_tiles * kTile; }
};

// Status codes shared with the C ABI.
enum : int32_t {
    kOk = 0,
    kErrArg = -1,
    kErrParse = -2,
    kErrRange = -3,
    kErrDevice = -4,
    kErrNoMem = -5,
    kErrNonFinite = -6,
    kErrCancelled = -7,
    kErrIO = -8,
    kErrTooLarge = -9,
};

// weights: one positive weight per clause (at most 2^53, total below 2^63), or null.
int32_t build_plan(int32_t n, const int32_t* lits, int64_t nlits, const int64_t* weights, HostPlan& plan,
                   std::string& err);
// DIMACS "p cnf", weighted "p wcnf n m top" (each clause led by its weight),
// or the header-less weighted form whose clauses are led by a weight or by
// "h" (hard: weight 1 + the total soft weight).  weights is left empty for
// plain CNF.
// The clause-side -> variable-side occurrence map on the host, by scanning
// each occurrence's clause row for its variable (the same rule as the
// device build); leaves c_slot empty when !slot_ok.
void build_slots(HostPlan& P);
int32_t read_dimacs(const char* path, int32_t& n, std::vector<int32_t>& lits, std::vector<int64_t>& weights,
                    std::string& err);

}  // namespace hms
