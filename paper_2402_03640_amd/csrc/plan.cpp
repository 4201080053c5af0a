// Instance plan builder.
//
// W (Section 4, network architecture) holds +1 where a variable appears in a
// clause, -1 where its negation does.  It is never stored dense: the plan keeps
// its nonzeros twice, clause-major for the scores f = tanh(x) W and
// variable-major for the transposed product W a of the backward pass.
//
// Canonical form of a clause: repeated literals count once; a variable that
// appears with both signs gets entry +1 - 1 = 0 and makes the clause always
// satisfied; an empty clause is always unsatisfied with score 0.
//
// Layout choices (all functions of the instance only, so every kernel schedule
// sums in the same order):
//  * clause rows sorted by (tautology flag, length descending, smallest
//    variable), cut into tiles of 64 rows stored column-major, padded to the
//    tile's longest row;
//  * variables renumbered by degree descending; a variable with more than
//    split_len entries (kSeg, or on dense instances the largest degree up to
//    kSplitDense) is split into ns = ceil(d / kSeg) segments, segment s holding
//    entries s, s + ns, s + 2 ns, ... of its list, and the segments' partial
//    sums are combined afterwards.  Interleaving puts consecutive entries in
//    neighbouring segment rows, so one column of a tile of a hot variable's
//    segments reads neighbouring adjoint entries;
//  * variable rows (segments first, then whole light variables) tiled the same
//    way; the entries of a row follow increasing clause-row index.
#include "plan.hpp"

#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <numeric>
#include <thread>
#include <utility>

namespace hms {

// ---- host buffers ---------------------------------------------------------
constexpr std::size_t kHuge = std::size_t(2) << 20;

void* build_alloc(std::size_t bytes) {
    if (bytes < kHuge) return ::operator new(bytes);
    const std::size_t len = (bytes + kHuge - 1) & ~(kHuge - 1);
    void* p = mmap(nullptr, len, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (p == MAP_FAILED) throw std::bad_alloc();
    (void)madvise(p, len, MADV_HUGEPAGE);  // a hint: without it the pages are 4 KiB
    return p;
}

void build_free(void* p, std::size_t bytes) noexcept {
    if (!p) return;
    if (bytes < kHuge) {
        ::operator delete(p);
        return;
    }
    (void)munmap(p, (bytes + kHuge - 1) & ~(kHuge - 1));
}

namespace {

struct Row {
    int64_t off;     // into the flat entry buffer
    int32_t len;
    int32_t orig;    // original clause index
    int32_t minvar;  // smallest new variable index of the row
    bool taut;
};

// ---- host threads ---------------------------------------------------------
// A build uses the host's hardware threads (at most 16), shared by the builds
// running at once in proportion to their literal counts (a large build next
// to small ones takes most of them: its latency is the longest), at least one
// each and one per 2^16 literals at most; the variable HIPMSAT_PLAN_THREADS
// sets the count instead (shared equally, with no size rule).  Every phase
// gives the same plan whatever the thread count: each is a fixed function of
// the instance.
std::atomic<int> g_active_builds{0};
std::atomic<int64_t> g_active_lits{0};

struct BuildSlot {
    int threads;
    int64_t lits;
    explicit BuildSlot(int64_t nlits) : lits(std::max<int64_t>(nlits, 1)) {
        const int active = g_active_builds.fetch_add(1) + 1;
        const int64_t all = g_active_lits.fetch_add(lits) + lits;
        const char* e = std::getenv("HIPMSAT_PLAN_THREADS");
        const int set = (e && *e) ? std::min(std::atoi(e), 64) : 0;
        if (set > 0) {
            threads = std::max(1, set / active);
        } else {
            const int cap = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
            const int64_t by_size = std::max<int64_t>(1, nlits >> 16);
            const int64_t share = (int64_t)((double)cap * (double)lits / (double)std::max<int64_t>(all, lits) + 0.5);
            threads = (int)std::max<int64_t>(1, std::min<int64_t>(share, by_size));
        }
    }
    ~BuildSlot() {
        g_active_lits.fetch_sub(lits);
        g_active_builds.fetch_sub(1);
    }
};

// Runs fn(t) for t = 0..T-1, thread 0 on the caller; an exception in any
// part is rethrown here after all have joined.
template <typename F>
void par(int T, const F& fn) {
    if (T <= 1) {
        fn(0);
        return;
    }
    std::vector<std::exception_ptr> ex((size_t)T);
    auto run = [&](int t) {
        try {
            fn(t);
        } catch (...) {
            ex[(size_t)t] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve((size_t)T - 1);
    try {
        for (int t = 1; t < T; ++t) th.emplace_back(run, t);
    } catch (...) {
        // could not start every thread: run the rest here
        for (int t = (int)th.size() + 1; t < T; ++t) run(t);
    }
    run(0);
    for (auto& x : th) x.join();
    for (auto& e : ex)
        if (e) std::rethrow_exception(e);
}

// Part t of T of [0, n): [lo, hi).
inline int64_t part_lo(int64_t n, int t, int T) { return (int64_t)((__int128)n * t / T); }

// Lay out rows (already ordered) into 64-row column-major tiles appended to
// tiles / ent; tiles fill in parallel at bases fixed beforehand.
template <typename LenFn, typename EntFn>
int32_t tile_rows(int T, int32_t nrows, LenFn len_of, EntFn ent_of, uint32_t pad, uint32_t flags,
                  PVec<TileDesc>& tiles, PVec<uint32_t>& ent, std::string& err) {
    const int32_t nt = (nrows + kTile - 1) / kTile;
    PVec<uint32_t> tlen((size_t)nt, 0);
    par(T, [&](int t) {
        for (int64_t k = part_lo(nt, t, T); k < part_lo(nt, t + 1, T); ++k) {
            uint32_t len = 0;
            const int32_t r1 = std::min<int32_t>(nrows, (int32_t)k * kTile + kTile);
            for (int32_t r = (int32_t)k * kTile; r < r1; ++r) len = std::max<uint32_t>(len, (uint32_t)len_of(r));
            tlen[(size_t)k] = len;
        }
    });
    const size_t t0 = tiles.size();
    uint64_t base = ent.size();
    tiles.reserve(t0 + (size_t)nt);
    for (int32_t k = 0; k < nt; ++k) {
        if (base + (uint64_t)tlen[(size_t)k] * kTile > 0xffffffffull) {
            err = "instance too large: more than 2^32 padded entries";
            return kErrTooLarge;
        }
        tiles.push_back(TileDesc{(uint32_t)base, tlen[(size_t)k],
                                 (uint32_t)std::min<int32_t>(kTile, nrows - k * kTile), flags});
        base += (uint64_t)tlen[(size_t)k] * kTile;
    }
    ent.resize((size_t)base, pad);
    par(T, [&](int t) {
        for (int64_t k = part_lo(nt, t, T); k < part_lo(nt, t + 1, T); ++k) {
            const TileDesc& d = tiles[t0 + (size_t)k];
            for (uint32_t q = 0; q < d.nreal; ++q) {
                const int32_t r = (int32_t)k * kTile + (int32_t)q;
                const int32_t L = len_of(r);
                for (int32_t c = 0; c < L; ++c) ent[d.base + (size_t)c * kTile + q] = ent_of(r, c);
            }
        }
    });
    return kOk;
}

// Canonical entries of the clauses in lits[b0, b1) (whole clauses), numbered
// from j0: a variable is emitted at its first appearance with its sign,
// unless it also appears negated (then the clause is a tautology).
struct Chunk {
    PVec<uint32_t> flat;  // original variable | sign
    PVec<Row> rows;       // off into this chunk's flat
    int32_t m_empty = 0, m_taut = 0, m_taut_dropped = 0;
    int64_t w_empty = 0;
};

void canonical_chunk(const int32_t* lits, int64_t b0, int64_t b1, int32_t j0, const int64_t* weights, Chunk& C) {
    constexpr int kShort = 16;  // clauses up to this length are deduplicated in registers
    PVec<uint64_t> key;  // longer ones: (variable, position) sorted
    PVec<uint64_t> emit; // (position, entry) of the emitted literals
    int64_t start = b0;
    int32_t j = j0;
    for (int64_t p = b0; p < b1; ++p) {
        if (lits[p] != 0) continue;
        const int k64 = (int)std::min<int64_t>(p - start, INT32_MAX);
        const int64_t off = (int64_t)C.flat.size();
        bool taut = false;
        if (p - start <= kShort) {
            // pairwise comparison
            const int k = k64;
            int32_t v[kShort];
            uint8_t sg[kShort];
            for (int q = 0; q < k; ++q) {
                v[q] = std::abs(lits[start + q]) - 1;
                sg[q] = lits[start + q] > 0 ? 1 : 2;
            }
            for (int q = 0; q < k; ++q) {
                bool first = true;
                uint8_t both = sg[q];
                for (int u = 0; u < k; ++u) {
                    if (v[u] != v[q]) continue;
                    if (u < q) first = false;
                    both |= sg[u];
                }
                if (!first) continue;
                if (both == 3) {
                    taut = true;
                    continue;
                }
                C.flat.push_back((uint32_t)v[q] | ((both & 2) ? kSign : 0u));
            }
        } else {
            // the same rule through a sort by (variable, position)
            const int64_t k = p - start;
            key.resize((size_t)k);
            for (int64_t q = 0; q < k; ++q) key[(size_t)q] = ((uint64_t)(std::abs(lits[start + q]) - 1) << 32) | (uint64_t)q;
            std::sort(key.begin(), key.end());
            emit.clear();
            for (int64_t g = 0; g < k;) {
                const uint32_t v = (uint32_t)(key[(size_t)g] >> 32);
                int64_t h = g;
                uint8_t both = 0;
                while (h < k && (uint32_t)(key[(size_t)h] >> 32) == v) {
                    both |= lits[start + (int64_t)(uint32_t)key[(size_t)h]] > 0 ? 1 : 2;
                    ++h;
                }
                if (both == 3) taut = true;
                else emit.push_back((key[(size_t)g] << 32) | (v | ((both & 2) ? kSign : 0u)));  // first position
                g = h;
            }
            std::sort(emit.begin(), emit.end());  // by position
            for (uint64_t e : emit) C.flat.push_back((uint32_t)e);
        }
        const int32_t len = (int32_t)((int64_t)C.flat.size() - off);
        if (p == start) {
            C.m_empty++;
            C.w_empty += weights ? weights[j] : 1;
        } else if (taut) {
            C.m_taut++;
            if (len == 0) C.m_taut_dropped++;
        }
        if (len > 0) C.rows.push_back(Row{off, len, j, 0, taut});
        ++j;
        start = p + 1;
    }
}

int32_t build_plan_impl(int32_t n, const int32_t* lits, int64_t nlits, const int64_t* weights, HostPlan& P,
                        std::string& err) {
    P = HostPlan{};
    if (n < 0 || nlits < 0 || (nlits > 0 && lits == nullptr)) {
        err = "bad arguments: n_vars < 0, n_lits < 0 or null literal array";
        return kErrArg;
    }
    if (n >= (int32_t)kIdx) {
        err = "too many variables";
        return kErrTooLarge;
    }
    if (nlits > 0 && lits[nlits - 1] != 0) {
        err = "last clause is not terminated by 0";
        return kErrParse;
    }
    BuildSlot slot(nlits);
    const int T = slot.threads;

    // ---- chunks of whole clauses; checks and counts per chunk ---------------
    PVec<int64_t> cb((size_t)T + 1, nlits);
    cb[0] = 0;
    for (int t = 1; t < T; ++t) {
        int64_t q = std::max(cb[(size_t)t - 1], part_lo(nlits, t, T));
        while (q < nlits && q > 0 && lits[q - 1] != 0) ++q;  // the next clause start
        cb[(size_t)t] = q;
    }
    PVec<int64_t> zeros((size_t)T, 0), nonzero((size_t)T, 0), bad((size_t)T, -1);
    par(T, [&](int t) {
        int64_t z = 0, nz = 0;  // counted in registers, stored once (no shared cache lines in the loop)
        for (int64_t p = cb[(size_t)t]; p < cb[(size_t)t + 1]; ++p) {
            const int32_t l = lits[p];
            if (l == 0) {
                ++z;
                continue;
            }
            if (l == INT32_MIN || std::abs(l) > n) {
                bad[(size_t)t] = p;  // the first one of the chunk
                return;
            }
            ++nz;
        }
        zeros[(size_t)t] = z;
        nonzero[(size_t)t] = nz;
    });
    for (int t = 0; t < T; ++t)
        if (bad[(size_t)t] >= 0) {
            const int64_t p = bad[(size_t)t];
            char buf[128];
            snprintf(buf, sizeof buf, "literal %d at position %lld is outside 1..%d", lits[p], (long long)p, n);
            err = buf;
            return kErrRange;
        }
    int64_t m = 0;
    PVec<int32_t> j0((size_t)T, 0);
    for (int t = 0; t < T; ++t) {
        if (m >= (int64_t)kIdx) break;
        j0[(size_t)t] = (int32_t)m;
        m += zeros[(size_t)t];
        P.lits_in += nonzero[(size_t)t];
    }
    if (m >= (int64_t)kIdx) {
        err = "too many clauses";
        return kErrTooLarge;
    }
    P.n = n;
    P.m = (int32_t)m;
    P.w_total = m;
    if (weights) {
        int64_t tot = 0;
        for (int64_t j = 0; j < m; ++j) {
            if (weights[j] <= 0 || weights[j] > ((int64_t)1 << 53) || tot > INT64_MAX - weights[j]) {
                err = "clause weights must be positive, at most 2^53, with a total below 2^63";
                return kErrArg;
            }
            tot += weights[j];
        }
        P.weighted = true;
        P.w_total = tot;
    }

    // ---- canonical clauses: W entries in order of first appearance --------
    PVec<uint32_t> flat;  // original variable | sign, then new variable | sign
    PVec<Row> rows;
    {
        PVec<Chunk> ch((size_t)T);
        par(T, [&](int t) { canonical_chunk(lits, cb[(size_t)t], cb[(size_t)t + 1], j0[(size_t)t], weights, ch[(size_t)t]); });
        PVec<int64_t> foff((size_t)T + 1, 0), roff((size_t)T + 1, 0);
        for (int t = 0; t < T; ++t) {
            const Chunk& c = ch[(size_t)t];
            foff[(size_t)t + 1] = foff[(size_t)t] + (int64_t)c.flat.size();
            roff[(size_t)t + 1] = roff[(size_t)t] + (int64_t)c.rows.size();
            P.m_empty += c.m_empty;
            P.m_taut += c.m_taut;
            P.m_taut_dropped += c.m_taut_dropped;
            P.w_empty += c.w_empty;
        }
        flat.resize((size_t)foff[(size_t)T]);
        rows.resize((size_t)roff[(size_t)T]);
        par(T, [&](int t) {
            Chunk& c = ch[(size_t)t];
            if (!c.flat.empty()) std::memcpy(&flat[(size_t)foff[(size_t)t]], c.flat.data(), c.flat.size() * 4);
            for (size_t i = 0; i < c.rows.size(); ++i) {
                Row r = c.rows[i];
                r.off += foff[(size_t)t];
                rows[(size_t)roff[(size_t)t] + i] = r;
            }
            PVec<uint32_t>().swap(c.flat);
        });
    }
    P.nnz = (int64_t)flat.size();

    // ---- variable order: degree descending, ties by original index -------
    PVec<int32_t> deg_orig((size_t)n, 0);
    if ((int64_t)T * n <= ((int64_t)1 << 26) && T > 1) {
        // per-thread histograms, then a sum over variable ranges
        std::vector<std::vector<int32_t>> h((size_t)T);
        par(T, [&](int t) {
            h[(size_t)t].assign((size_t)n, 0);
            for (int64_t e = part_lo(P.nnz, t, T); e < part_lo(P.nnz, t + 1, T); ++e) h[(size_t)t][flat[(size_t)e] & kIdx]++;
        });
        par(T, [&](int t) {
            for (int64_t i = part_lo(n, t, T); i < part_lo(n, t + 1, T); ++i) {
                int32_t d = 0;
                for (int u = 0; u < T; ++u) d += h[(size_t)u][(size_t)i];
                deg_orig[(size_t)i] = d;
            }
        });
    } else {
        for (uint32_t e : flat) deg_orig[e & kIdx]++;
    }
    // counting sort: degree descending, ties by original index (stable)
    {
        int32_t maxd = 0;
        for (int32_t i = 0; i < n; ++i) maxd = std::max(maxd, deg_orig[i]);
        PVec<int64_t> start((size_t)maxd + 2, 0);
        for (int32_t i = 0; i < n; ++i) start[(size_t)(maxd - deg_orig[i]) + 1]++;
        for (int32_t d = 0; d <= maxd; ++d) start[d + 1] += start[d];
        P.var_old.resize((size_t)n);
        for (int32_t i = 0; i < n; ++i) P.var_old[start[(size_t)(maxd - deg_orig[i])]++] = i;
    }
    P.var_new.assign((size_t)n, 0);
    P.degree.assign((size_t)n, 0);
    int32_t n_long = 0;  // variables with more than kSeg entries
    for (int32_t i = 0; i < n; ++i) {
        P.var_new[P.var_old[i]] = i;
        P.degree[i] = deg_orig[P.var_old[i]];
        if (P.degree[i] > 0) P.n_act = i + 1;
        if (P.degree[i] > kSeg) n_long = i + 1;
    }
    // A split row costs its segments' partial sums and a combine pass.  When a
    // quarter or more of the variables are long (dense uniform instances,
    // where nearly every row is) and none exceeds kSplitDense, no row is
    // split: each lane sums its whole row.  Otherwise rows above kSeg are.
    const int32_t maxd = n > 0 ? P.degree[0] : 0;
    P.split_len = ((int64_t)n_long * 4 >= (int64_t)P.n_act && n_long > 0 && maxd <= kSplitDense) ? maxd : kSeg;
    while (P.n_heavy < n && P.degree[P.n_heavy] > P.split_len) ++P.n_heavy;
    // from here on the flat entries hold the new variable index, and each row
    // knows its smallest one
    const int64_t nr = (int64_t)rows.size();
    par(T, [&](int t) {
        for (int64_t e = part_lo(P.nnz, t, T); e < part_lo(P.nnz, t + 1, T); ++e)
            flat[(size_t)e] = (uint32_t)P.var_new[flat[(size_t)e] & kIdx] | (flat[(size_t)e] & kSign);
    });
    par(T, [&](int t) {
        for (int64_t i = part_lo(nr, t, T); i < part_lo(nr, t + 1, T); ++i) {
            Row& r = rows[(size_t)i];
            int32_t mv = INT32_MAX;
            for (int32_t c = 0; c < r.len; ++c) mv = std::min(mv, (int32_t)(flat[(size_t)r.off + c] & kIdx));
            r.minvar = mv;
        }
    });

    // ---- clause rows: plain rows by length desc, then tautological rows; ---
    // within a length, by the smallest (hottest) new variable index, so that
    // the clauses of a frequent variable sit together and its transposed row
    // reads neighbouring adjoint entries; ties keep the clause order.  A
    // least-significant-digit radix sort on (length class, smallest
    // variable), 11 bits a pass, each pass a stable scatter with per-thread
    // counts; then the rows and their entries are gathered into that order
    // once.
    {
        int32_t maxl = 0;
        for (const Row& r : rows) maxl = std::max(maxl, r.len);
        int vbits = 1;
        while (vbits < 31 && ((int64_t)1 << vbits) < (int64_t)n) ++vbits;
        PVec<uint64_t> key((size_t)nr), key2((size_t)nr);
        PVec<int32_t> ord((size_t)nr), ord2((size_t)nr);
        uint64_t kmax = 0;
        par(T, [&](int t) {
            for (int64_t i = part_lo(nr, t, T); i < part_lo(nr, t + 1, T); ++i) {
                const Row& r = rows[(size_t)i];
                // class: plain rows of length maxl - c for c <= maxl, then tautologies likewise
                const uint64_t cls = (uint64_t)((r.taut ? maxl + 1 : 0) + (maxl - r.len));
                key[(size_t)i] = (cls << vbits) | (uint64_t)r.minvar;
                ord[(size_t)i] = (int32_t)i;
            }
        });
        kmax = ((uint64_t)(2 * (maxl + 1)) << vbits);
        constexpr int kDigit = 11;
        constexpr int kBins = 1 << kDigit;
        std::vector<std::vector<int64_t>> cnt((size_t)T);
        for (int shift = 0; shift < 64 && (kmax >> shift) != 0; shift += kDigit) {
            par(T, [&](int t) {
                std::vector<int64_t>& c = cnt[(size_t)t];
                c.assign(kBins, 0);
                for (int64_t i = part_lo(nr, t, T); i < part_lo(nr, t + 1, T); ++i)
                    c[(key[(size_t)i] >> shift) & (kBins - 1)]++;
            });
            int64_t o = 0;
            for (int d = 0; d < kBins; ++d)
                for (int t = 0; t < T; ++t) {
                    const int64_t c = cnt[(size_t)t][d];
                    cnt[(size_t)t][d] = o;  // this thread's first slot for digit d
                    o += c;
                }
            par(T, [&](int t) {
                std::vector<int64_t>& c = cnt[(size_t)t];
                for (int64_t i = part_lo(nr, t, T); i < part_lo(nr, t + 1, T); ++i) {
                    const int64_t q = c[(key[(size_t)i] >> shift) & (kBins - 1)]++;
                    key2[(size_t)q] = key[(size_t)i];
                    ord2[(size_t)q] = ord[(size_t)i];
                }
            });
            key.swap(key2);
            ord.swap(ord2);
        }
        PVec<uint64_t>().swap(key);
        PVec<uint64_t>().swap(key2);
        PVec<int64_t> psum((size_t)T + 1, 0);
        par(T, [&](int t) {
            int64_t s = 0;
            for (int64_t r = part_lo(nr, t, T); r < part_lo(nr, t + 1, T); ++r) s += rows[(size_t)ord[(size_t)r]].len;
            psum[(size_t)t + 1] = s;
        });
        for (int t = 0; t < T; ++t) psum[(size_t)t + 1] += psum[(size_t)t];
        PVec<Row> sorted((size_t)nr);
        PVec<uint32_t> flat2(flat.size());
        par(T, [&](int t) {
            int64_t o = psum[(size_t)t];
            constexpr int64_t kAhead = 16;  // rows fetched ahead of the copy
            const int64_t r1 = part_lo(nr, t + 1, T);
            for (int64_t r = part_lo(nr, t, T); r < r1; ++r) {
                if (r + kAhead < r1) {
                    const Row& f = rows[(size_t)ord[(size_t)(r + kAhead)]];
                    __builtin_prefetch(&f);
                    __builtin_prefetch(&flat[(size_t)f.off]);
                }
                Row R = rows[(size_t)ord[(size_t)r]];
                std::memcpy(&flat2[(size_t)o], &flat[(size_t)R.off], (size_t)R.len * 4);
                R.off = o;
                o += R.len;
                sorted[(size_t)r] = R;
            }
        });
        rows.swap(sorted);
        flat.swap(flat2);
    }
    int32_t n_plain = 0;
    while (n_plain < (int32_t)rows.size() && !rows[n_plain].taut) ++n_plain;
    int32_t n_tr = (int32_t)rows.size() - n_plain;
    const uint32_t cpad = (uint32_t)n;  // dummy variable whose relaxed value stays -0.0
    int32_t rc;
    rc = tile_rows(T, n_plain, [&](int32_t r) { return rows[r].len; },
                   [&](int32_t r, int32_t c) { return flat[rows[r].off + c]; }, cpad, 0u, P.c_tile, P.c_ent, err);
    if (rc) return rc;
    rc = tile_rows(T, n_tr, [&](int32_t r) { return rows[n_plain + r].len; },
                   [&](int32_t r, int32_t c) { return flat[rows[n_plain + r].off + c]; }, cpad, 1u, P.c_tile,
                   P.c_ent, err);
    if (rc) return rc;
    P.c_tiles = (int32_t)P.c_tile.size();
    if ((int64_t)P.c_tiles * kTile + 1 >= (int64_t)kIdx) {
        err = "too many clause rows";
        return kErrTooLarge;
    }
    P.mk = (int32_t)rows.size();
    // kernel row index of each canonical row
    PVec<int32_t> krow(rows.size());
    P.c_row_orig.assign((size_t)P.c_tiles * kTile, -1);
    {
        const int32_t tp = (n_plain + kTile - 1) / kTile;
        if (weights) P.c_w.assign((size_t)P.c_tiles * kTile, 0);
        par(T, [&](int t) {
            for (int64_t r = part_lo(nr, t, T); r < part_lo(nr, t + 1, T); ++r) {
                const int32_t k = r < n_plain ? (int32_t)r : tp * kTile + (int32_t)(r - n_plain);
                krow[(size_t)r] = k;
                P.c_row_orig[(size_t)k] = rows[(size_t)r].orig;
                if (weights) P.c_w[(size_t)k] = weights[rows[(size_t)r].orig];
            }
        });
    }

    // ---- variable-major occurrence lists (clause rows ascending) ----------
    PVec<int64_t> voff((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) voff[i + 1] = voff[i] + P.degree[i];
    PVec<uint32_t> occ((size_t)P.nnz);
    {
        // Two stable scatters with few write streams each: (1) (variable,
        // kernel row) pairs into blocks of 1024 consecutive variables, each
        // thread taking a range of rows and writing after the threads before
        // it, (2) each block into its variables' lists.  Rows are visited in
        // increasing kernel-row order, so every list ends in increasing
        // kernel-row order.
        constexpr int kShift = 10;
        const int32_t nblk = (n >> kShift) + 1;
        PVec<int64_t> bstart((size_t)nblk + 1, 0);
        for (int32_t b = 0; b < nblk; ++b)
            bstart[b + 1] = voff[std::min<int64_t>((int64_t)(b + 1) << kShift, n)];
        PVec<uint64_t> pairs((size_t)P.nnz);  // variable << 32 | (row | sign)
        std::vector<std::vector<int64_t>> cnt((size_t)T);
        par(T, [&](int t) {
            cnt[(size_t)t].assign((size_t)nblk, 0);
            for (int64_t r = part_lo(nr, t, T); r < part_lo(nr, t + 1, T); ++r) {
                const Row& R = rows[(size_t)r];
                for (int32_t c = 0; c < R.len; ++c) cnt[(size_t)t][(flat[(size_t)R.off + c] & kIdx) >> kShift]++;
            }
        });
        for (int32_t b = 0; b < nblk; ++b) {
            int64_t o = bstart[b];
            for (int t = 0; t < T; ++t) {
                const int64_t c = cnt[(size_t)t][b];
                cnt[(size_t)t][b] = o;  // this thread's first slot in block b
                o += c;
            }
        }
        par(T, [&](int t) {
            std::vector<int64_t>& fill = cnt[(size_t)t];
            for (int64_t r = part_lo(nr, t, T); r < part_lo(nr, t + 1, T); ++r) {
                const Row& R = rows[(size_t)r];
                for (int32_t c = 0; c < R.len; ++c) {
                    const uint32_t e = flat[(size_t)R.off + c];
                    const uint32_t v = e & kIdx;
                    pairs[(size_t)fill[v >> kShift]++] = ((uint64_t)v << 32) | (uint32_t)krow[(size_t)r] | (e & kSign);
                }
            }
        });
        par(T, [&](int t) {
            PVec<int64_t> fill;
            for (int64_t b = part_lo(nblk, t, T); b < part_lo(nblk, t + 1, T); ++b) {
                const int64_t v0 = b << kShift, v1 = std::min<int64_t>((b + 1) << kShift, n);
                fill.assign(voff.begin() + v0, voff.begin() + std::max(v0, v1));
                for (int64_t p = bstart[(size_t)b]; p < bstart[(size_t)b + 1]; ++p) {
                    const uint64_t q = pairs[(size_t)p];
                    occ[(size_t)fill[(size_t)((int64_t)(q >> 32) - v0)]++] = (uint32_t)q;
                }
            }
        });
    }

    // ---- segments of heavy variables ---------------------------------------
    struct Seg {
        int32_t var, idx, len, stride;
        int64_t off;
    };
    PVec<Seg> segs;
    P.seg_first.assign((size_t)P.n_heavy + 1, 0);
    for (int32_t h = 0; h < P.n_heavy; ++h) {
        int32_t d = P.degree[h];
        int32_t ns = (d + kSeg - 1) / kSeg;
        P.max_segs = std::max(P.max_segs, ns);
        if (ns > kWideSegs) P.n_heavy_wide = h + 1;
        P.seg_first[h + 1] = P.seg_first[h] + ns;
        for (int32_t s = 0; s < ns; ++s) segs.push_back(Seg{h, s, (d - s + ns - 1) / ns, ns, voff[h] + s});
    }
    // rows in (variable, segment) order: a variable's partial sums sit side by
    // side for the combine, and its segments' lengths differ by at most one
    P.seg_rows = (int32_t)segs.size();
    P.seg_row.resize((size_t)P.seg_rows);
    std::iota(P.seg_row.begin(), P.seg_row.end(), 0);
    const uint32_t vpad = (uint32_t)P.a_zero_row();
    rc = tile_rows(T, P.seg_rows, [&](int32_t r) { return segs[r].len; },
                   [&](int32_t r, int32_t c) { return occ[segs[r].off + (int64_t)c * segs[r].stride]; }, vpad, 0u,
                   P.v_tile, P.v_ent, err);
    if (rc) return rc;
    P.seg_tiles = (int32_t)P.v_tile.size();
    int32_t n_light = P.n_act - P.n_heavy;
    rc = tile_rows(T, n_light, [&](int32_t r) { return P.degree[P.n_heavy + r]; },
                   [&](int32_t r, int32_t c) { return occ[voff[P.n_heavy + r] + c]; }, vpad, 0u,
                   P.v_tile, P.v_ent, err);
    if (rc) return rc;
    P.v_tiles = (int32_t)P.v_tile.size();
    // the slot schedules index the variable side with 31 bits
    P.slot_ok = P.v_ent.size() < (size_t)kIdx;
    P.build_threads = T;
    return kOk;
}

}  // namespace

void build_slots(HostPlan& P) {
    P.c_slot.clear();
    if (!P.slot_ok) return;
    P.c_slot.assign(P.c_ent.size(), kNoSlot);
    const uint32_t vpad = (uint32_t)P.a_zero_row();
    for (int32_t t = 0; t < P.v_tiles; ++t) {
        const TileDesc& d = P.v_tile[(size_t)t];
        for (uint32_t q = 0; q < d.nreal; ++q) {
            const int32_t row = t * kTile + (int32_t)q;
            // variable of the row: a heavy variable's segments, or a light row
            int32_t v;
            if (row < P.seg_rows)
                v = (int32_t)(std::upper_bound(P.seg_first.begin(), P.seg_first.end(), row) - P.seg_first.begin()) - 1;
            else
                v = P.n_heavy + (row - P.seg_tiles * kTile);
            for (uint32_t c = 0; c < d.len; ++c) {
                const uint32_t vpos = d.base + c * kTile + q;
                const uint32_t e = P.v_ent[vpos];
                if (e == vpad) continue;
                const uint32_t j = e & kIdx;
                const TileDesc& cd = P.c_tile[j / kTile];
                for (uint32_t cc = 0; cc < cd.len; ++cc) {
                    const uint32_t cpos = cd.base + cc * kTile + j % kTile;
                    if ((P.c_ent[cpos] & kIdx) == (uint32_t)v) {
                        P.c_slot[cd.base + (j % kTile) * cd.len + cc] = vpos | (e & kSign);  // row-major in the tile
                        break;
                    }
                }
            }
        }
    }
}

int32_t build_plan(int32_t n, const int32_t* lits, int64_t nlits, const int64_t* weights, HostPlan& P,
                   std::string& err) {
    try {
        return build_plan_impl(n, lits, nlits, weights, P, err);
    } catch (const std::bad_alloc&) {
        P = HostPlan{};
        err = "host allocation failed while building the plan";
        return kErrNoMem;
    } catch (const std::exception& e) {
        P = HostPlan{};
        err = std::string("plan build failed: ") + e.what();
        return kErrNoMem;
    }
}

int32_t read_dimacs(const char* path, int32_t& n, std::vector<int32_t>& lits, std::vector<int64_t>& weights,
                    std::string& err) {
    FILE* f = fopen(path, "rb");
    if (!f) {
        err = std::string("cannot open ") + path + ": " + strerror(errno);
        return kErrIO;
    }
    std::string buf;
    {
        char chunk[1 << 16];
        size_t got;
        while ((got = fread(chunk, 1, sizeof chunk, f)) > 0) buf.append(chunk, got);
    }
    fclose(f);
    n = -1;
    lits.clear();
    weights.clear();
    enum { kCnf, kWcnf, kWcnfNoHeader } mode = kCnf;
    bool header = false, in_clause = false, any_hard = false;
    int64_t soft_total = 0;
    int32_t maxv = 0;
    const char* s = buf.c_str();
    const char* end = s + buf.size();
    while (s < end) {
        // one line
        const char* eol = (const char*)memchr(s, '\n', (size_t)(end - s));
        if (!eol) eol = end;
        std::string line(s, eol);
        s = eol + 1;
        size_t q = line.find_first_not_of(" \t\r");
        if (q == std::string::npos) continue;
        const char c0 = line[q];
        if (c0 == 'c' || c0 == '%') continue;
        if (c0 == 'p') {
            char fmt[16] = {0};
            long long nv = -1, nc = -1;
            if (header || sscanf(line.c_str() + q, "p %15s %lld %lld", fmt, &nv, &nc) != 3 || nv < 0 || nc < 0 ||
                nv >= (long long)kIdx || (strcmp(fmt, "cnf") != 0 && strcmp(fmt, "wcnf") != 0)) {
                err = "bad problem line";
                return kErrParse;
            }
            header = true;
            mode = strcmp(fmt, "wcnf") == 0 ? kWcnf : kCnf;
            n = (int32_t)nv;
            continue;
        }
        if (!header && !in_clause && c0 == 'h') mode = kWcnfNoHeader;
        const char* t = line.c_str() + q;
        while (true) {
            while (*t == ' ' || *t == '\t' || *t == '\r') ++t;
            if (*t == 0) break;
            if (!in_clause && mode != kCnf) {
                // the clause's weight, or "h" for a hard clause
                if (*t == 'h' && mode == kWcnfNoHeader) {
                    weights.push_back(-1);
                    any_hard = true;
                    ++t;
                } else {
                    char* e = nullptr;
                    errno = 0;
                    long long w = strtoll(t, &e, 10);
                    if (e == t || errno || w <= 0) {
                        err = "bad clause weight";
                        return kErrParse;
                    }
                    weights.push_back(w);
                    if (soft_total > INT64_MAX - w) {
                        err = "clause weights overflow";
                        return kErrParse;
                    }
                    soft_total += w;
                    t = e;
                }
                in_clause = true;
                if (*t != ' ' && *t != '\t' && *t != 0 && *t != '\r') {
                    err = "bad clause weight";
                    return kErrParse;
                }
                continue;
            }
            char* e = nullptr;
            errno = 0;
            long v = strtol(t, &e, 10);
            if (e == t || errno) {
                err = "bad literal token";
                return kErrParse;
            }
            t = e;
            if (v < -(long)kIdx || v > (long)kIdx) {
                err = "literal out of range";
                return kErrRange;
            }
            lits.push_back((int32_t)v);
            in_clause = v != 0;
            if (v != 0) maxv = std::max<int32_t>(maxv, (int32_t)std::labs(v));
        }
    }
    if (in_clause) {
        err = "last clause is not terminated by 0";
        return kErrParse;
    }
    if (any_hard) {
        // a hard clause outweighs every soft clause together
        if (soft_total == INT64_MAX) {
            err = "clause weights overflow";
            return kErrParse;
        }
        for (int64_t& w : weights)
            if (w < 0) w = soft_total + 1;
    }
    if (n < 0) n = maxv;
    return kOk;
}

}  // namespace hms
