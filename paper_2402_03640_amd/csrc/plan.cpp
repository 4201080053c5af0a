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

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

namespace hms {

namespace {

struct Row {
    int64_t off;     // into the flat entry buffer
    int32_t len;
    int32_t orig;    // original clause index
    int32_t minvar;  // smallest new variable index of the row
    bool taut;
};

// Lay out rows (already ordered) into 64-row column-major tiles.
template <typename LenFn, typename EntFn>
int32_t tile_rows(int32_t nrows, LenFn len_of, EntFn ent_of,
                  uint32_t pad, uint32_t flags, std::vector<TileDesc>& tiles,
                  std::vector<uint32_t>& ent, std::string& err) {
    {
        // room for every tile up front (no regrowth)
        uint64_t total = ent.size();
        for (int32_t t0 = 0; t0 < nrows; t0 += kTile) {
            uint32_t len = 0;
            for (int32_t q = t0; q < std::min<int32_t>(nrows, t0 + kTile); ++q)
                len = std::max<uint32_t>(len, (uint32_t)len_of(q));
            total += (uint64_t)len * kTile;
        }
        if (total > 0xffffffffull) {
            err = "instance too large: more than 2^32 padded entries";
            return kErrTooLarge;
        }
        ent.reserve(total);
        tiles.reserve(tiles.size() + (nrows + kTile - 1) / kTile);
    }
    for (int32_t t0 = 0; t0 < nrows; t0 += kTile) {
        int32_t nreal = std::min<int32_t>(kTile, nrows - t0);
        uint32_t len = 0;
        for (int32_t q = 0; q < nreal; ++q) len = std::max<uint32_t>(len, (uint32_t)len_of(t0 + q));
        uint64_t base = ent.size();
        if (base + (uint64_t)len * kTile > 0xffffffffull) {
            err = "instance too large: more than 2^32 padded entries";
            return kErrTooLarge;
        }
        TileDesc d{(uint32_t)base, len, (uint32_t)nreal, flags};
        tiles.push_back(d);
        ent.resize(base + (size_t)len * kTile, pad);
        for (int32_t q = 0; q < nreal; ++q) {
            int32_t L = len_of(t0 + q);
            for (int32_t c = 0; c < L; ++c) ent[base + (size_t)c * kTile + q] = ent_of(t0 + q, c);
        }
    }
    return kOk;
}

}  // namespace

int32_t build_plan(int32_t n, const int32_t* lits, int64_t nlits, const int64_t* weights, HostPlan& P,
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
    int64_t m = 0;
    for (int64_t p = 0; p < nlits; ++p) {
        int32_t l = lits[p];
        if (l == 0) {
            ++m;
            continue;
        }
        if (l == INT32_MIN || std::abs(l) > n) {
            char buf[128];
            snprintf(buf, sizeof buf, "literal %d at position %lld is outside 1..%d", l, (long long)p, n);
            err = buf;
            return kErrRange;
        }
        P.lits_in++;
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
    std::vector<uint32_t> flat;          // original variable | sign
    flat.reserve((size_t)P.lits_in);
    std::vector<Row> rows;
    rows.reserve((size_t)m);
    std::vector<int64_t> stamp((size_t)n + 1, -1);
    std::vector<uint8_t> seen((size_t)n + 1, 0);   // bit0 positive, bit1 negative, bit2 emitted
    int64_t start = 0;
    int32_t j = 0;
    constexpr int kShort = 16;  // clauses up to this length are deduplicated in registers
    for (int64_t p = 0; p < nlits; ++p) {
        if (lits[p] != 0) continue;
        bool taut = false;
        if (p - start <= kShort) {
            // the same rule by pairwise comparison: a variable is emitted at its
            // first appearance with its sign, unless it also appears negated
            const int k = (int)(p - start);
            int32_t v[kShort];
            uint8_t sg[kShort];
            for (int q = 0; q < k; ++q) {
                v[q] = std::abs(lits[start + q]) - 1;
                sg[q] = lits[start + q] > 0 ? 1 : 2;
            }
            const int64_t off = (int64_t)flat.size();
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
                flat.push_back((uint32_t)v[q] | ((both & 2) ? kSign : 0u));
            }
            const int32_t len = (int32_t)((int64_t)flat.size() - off);
            if (p == start) {
                P.m_empty++;
                P.w_empty += weights ? weights[j] : 1;
            } else if (taut) {
                P.m_taut++;
                if (len == 0) P.m_taut_dropped++;
            }
            if (len > 0) rows.push_back(Row{off, len, j, 0, taut});
            ++j;
            start = p + 1;
            continue;
        }
        for (int64_t q = start; q < p; ++q) {
            int32_t v = std::abs(lits[q]) - 1;
            if (stamp[v] != j) {
                stamp[v] = j;
                seen[v] = 0;
            }
            seen[v] |= lits[q] > 0 ? 1 : 2;
        }
        int64_t off = (int64_t)flat.size();
        for (int64_t q = start; q < p; ++q) {
            int32_t v = std::abs(lits[q]) - 1;
            if (seen[v] & 4) continue;
            seen[v] |= 4;
            if ((seen[v] & 3) == 3) {
                taut = true;
                continue;
            }
            flat.push_back((uint32_t)v | ((seen[v] & 2) ? kSign : 0u));
        }
        int32_t len = (int32_t)((int64_t)flat.size() - off);
        if (p == start) {
            P.m_empty++;
            P.w_empty += weights ? weights[j] : 1;
        } else if (taut) {
            P.m_taut++;
            if (len == 0) P.m_taut_dropped++;
        }
        if (len > 0) rows.push_back(Row{off, len, j, 0, taut});
        ++j;
        start = p + 1;
    }
    P.nnz = (int64_t)flat.size();

    // ---- variable order: degree descending, ties by original index -------
    std::vector<int32_t> deg_orig((size_t)n, 0);
    for (uint32_t e : flat) deg_orig[e & kIdx]++;
    // counting sort: degree descending, ties by original index (stable)
    {
        int32_t maxd = 0;
        for (int32_t i = 0; i < n; ++i) maxd = std::max(maxd, deg_orig[i]);
        std::vector<int64_t> start((size_t)maxd + 2, 0);
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
    // from here on the flat entries hold the new variable index
    for (uint32_t& e : flat) e = (uint32_t)P.var_new[e & kIdx] | (e & kSign);

    // ---- clause rows: plain rows by length desc, then tautological rows; ---
    // within a length, by the smallest (hottest) new variable index, so that
    // the clauses of a frequent variable sit together and its transposed row
    // reads neighbouring adjoint entries.
    for (Row& r : rows) {
        int32_t mv = INT32_MAX;
        for (int32_t c = 0; c < r.len; ++c) mv = std::min(mv, (int32_t)(flat[r.off + c] & kIdx));
        r.minvar = mv;
    }
    // stable two-pass counting sort of row indices: by smallest variable,
    // then by (tautology flag, length descending); then the rows and their
    // entries are gathered into that order once, so every later pass reads
    // them sequentially
    {
        const size_t nr = rows.size();
        int32_t maxl = 0;
        for (const Row& r : rows) maxl = std::max(maxl, r.len);
        // bucket b: plain rows of length maxl - b for b <= maxl, then tautologies likewise
        const size_t nb = 2 * ((size_t)maxl + 1);
        std::vector<uint32_t> bucket_of(nr);
        std::vector<int64_t> cnt((size_t)n + 2, 0), c2(nb + 1, 0);
        for (size_t i = 0; i < nr; ++i) {
            const Row& r = rows[i];
            bucket_of[i] = (uint32_t)((r.taut ? maxl + 1 : 0) + (maxl - r.len));
            cnt[(size_t)r.minvar + 1]++;
            c2[bucket_of[i] + 1]++;
        }
        for (int32_t v = 0; v <= n; ++v) cnt[v + 1] += cnt[v];
        for (size_t b = 0; b < nb; ++b) c2[b + 1] += c2[b];
        std::vector<int32_t> tmp(nr), ord(nr);
        for (size_t i = 0; i < nr; ++i) tmp[cnt[rows[i].minvar]++] = (int32_t)i;
        for (int32_t i : tmp) ord[c2[bucket_of[i]]++] = i;
        std::vector<Row> sorted(nr);
        std::vector<uint32_t> flat2(flat.size());
        int64_t o = 0;
        constexpr size_t kAhead = 16;  // rows fetched ahead of the copy
        for (size_t r = 0; r < nr; ++r) {
            if (r + kAhead < nr) {
                const Row& f = rows[ord[r + kAhead]];
                __builtin_prefetch(&f);
                __builtin_prefetch(&flat[f.off]);
            }
            Row R = rows[ord[r]];
            std::memcpy(&flat2[o], &flat[R.off], (size_t)R.len * 4);
            R.off = o;
            o += R.len;
            sorted[r] = R;
        }
        rows.swap(sorted);
        flat.swap(flat2);
    }
    int32_t n_plain = 0;
    while (n_plain < (int32_t)rows.size() && !rows[n_plain].taut) ++n_plain;
    int32_t n_tr = (int32_t)rows.size() - n_plain;
    const uint32_t cpad = (uint32_t)n;  // dummy variable whose relaxed value stays -0.0
    int32_t rc;
    rc = tile_rows(n_plain, [&](int32_t r) { return rows[r].len; },
                   [&](int32_t r, int32_t c) { return flat[rows[r].off + c]; }, cpad, 0u, P.c_tile, P.c_ent, err);
    if (rc) return rc;
    rc = tile_rows(n_tr, [&](int32_t r) { return rows[n_plain + r].len; },
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
    std::vector<int32_t> krow(rows.size());
    P.c_row_orig.assign((size_t)P.c_tiles * kTile, -1);
    {
        int32_t tp = (n_plain + kTile - 1) / kTile;
        for (int32_t r = 0; r < n_plain; ++r) krow[r] = r;
        for (int32_t r = 0; r < n_tr; ++r) krow[n_plain + r] = tp * kTile + r;
        for (size_t r = 0; r < rows.size(); ++r) P.c_row_orig[krow[r]] = rows[r].orig;
        if (weights) {
            P.c_w.assign((size_t)P.c_tiles * kTile, 0);
            for (size_t r = 0; r < rows.size(); ++r) P.c_w[krow[r]] = weights[rows[r].orig];
        }
    }

    // ---- variable-major occurrence lists (clause rows ascending) ----------
    std::vector<int64_t> voff((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) voff[i + 1] = voff[i] + P.degree[i];
    std::vector<uint32_t> occ((size_t)P.nnz);
    {
        // Two passes, each with few write streams: (1) scatter (variable,
        // kernel row) pairs into blocks of 1024 consecutive variables, (2)
        // scatter each block into its variables' lists.  Rows are visited in
        // increasing kernel-row order and both passes are stable, so every
        // list ends in increasing kernel-row order.
        constexpr int kShift = 10;
        const int32_t nblk = (n >> kShift) + 1;
        std::vector<int64_t> bstart((size_t)nblk + 1, 0);
        for (int32_t b = 0; b < nblk; ++b)
            bstart[b + 1] = voff[std::min<int64_t>((int64_t)(b + 1) << kShift, n)];
        std::vector<uint64_t> pairs((size_t)P.nnz);  // variable << 32 | (row | sign)
        std::vector<int64_t> bfill(bstart.begin(), bstart.end() - 1);
        for (size_t r = 0; r < rows.size(); ++r) {
            const Row& R = rows[r];
            for (int32_t c = 0; c < R.len; ++c) {
                const uint32_t e = flat[R.off + c];
                const uint32_t v = e & kIdx;
                pairs[bfill[v >> kShift]++] = ((uint64_t)v << 32) | (uint32_t)krow[r] | (e & kSign);
            }
        }
        std::vector<int64_t> fill(voff.begin(), voff.end() - 1);
        for (const uint64_t q : pairs) occ[fill[q >> 32]++] = (uint32_t)q;
    }

    // ---- segments of heavy variables ---------------------------------------
    struct Seg {
        int32_t var, idx, len, stride;
        int64_t off;
    };
    std::vector<Seg> segs;
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
    rc = tile_rows(P.seg_rows, [&](int32_t r) { return segs[r].len; },
                   [&](int32_t r, int32_t c) { return occ[segs[r].off + (int64_t)c * segs[r].stride]; }, vpad, 0u, P.v_tile,
                   P.v_ent, err);
    if (rc) return rc;
    P.seg_tiles = (int32_t)P.v_tile.size();
    int32_t n_light = P.n_act - P.n_heavy;
    rc = tile_rows(n_light, [&](int32_t r) { return P.degree[P.n_heavy + r]; },
                   [&](int32_t r, int32_t c) { return occ[voff[P.n_heavy + r] + c]; }, vpad, 0u,
                   P.v_tile, P.v_ent, err);
    if (rc) return rc;
    P.v_tiles = (int32_t)P.v_tile.size();
    return kOk;
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
