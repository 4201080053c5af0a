// Solve-loop kernels for gfx950 (wave64).  See kernels.hpp for the layout.
//
// Summation order contract: the score of a clause is summed over its entries
// in plan order, and the transposed sum of a variable row over its entries in
// plan order, one lane per (row, restart), whatever the schedule.  Heavy rows
// are summed per segment, and segment partials are combined by a fixed tree
// (64 or 1024 slots, chosen by the instance).  Hence x, m, v and every count are bitwise independent of the
// schedule and of R; only the FP64 loss total depends on the schedule's unit
// size.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.hpp"

namespace hms {

const Schedule kSchedules[kNumSchedules + 1] = {
    {0, 0, 0, 0, 0},                                                                         // 0: automatic
    {1, 1, 1, 0, 0},  {2, 1, 1, 0, 0},  {4, 1, 1, 0, 0},  {8, 1, 1, 0, 0},  {8, 1, 2, 0, 0},   // 1..5
    {16, 1, 1, 0, 0}, {16, 1, 2, 0, 0}, {16, 1, 4, 0, 0}, {32, 1, 2, 0, 0}, {32, 1, 4, 0, 0},  // 6..10
    {64, 1, 1, 0, 0}, {64, 1, 2, 0, 0}, {64, 1, 4, 0, 0}, {64, 1, 8, 0, 0}, {16, 4, 1, 0, 0},  // 11..15
    {16, 4, 2, 0, 0}, {32, 2, 2, 0, 0}, {32, 2, 4, 0, 0}, {64, 2, 2, 0, 0}, {64, 2, 4, 0, 0},  // 16..20
    {64, 4, 1, 0, 0}, {64, 4, 2, 0, 0}, {1, 1, 1, 1, 1},  {2, 1, 1, 1, 2},  {4, 1, 1, 1, 3},   // 21..25
    {2, 4, 1, 0, 0},  {4, 2, 1, 0, 0},  {8, 1, 4, 0, 0},                                      // 26..28
    {1, 2, 1, 1, 27}, {1, 4, 1, 1, 26}, {2, 4, 1, 1, 26}, {4, 2, 1, 1, 27},                  // 29..32
    {4, 4, 1, 0, 0},  {8, 4, 1, 0, 0},  {8, 2, 1, 0, 0},                                      // 33..35
    {1, 1, 1, 0, 0, 2}, {1, 1, 1, 1, 36, 2},                                                  // 36..37
    {2, 1, 1, 0, 0, 1, 16}, {4, 1, 1, 0, 0, 1, 16}, {1, 1, 1, 0, 0, 2, 16},                    // 38..40
    {1, 1, 1, 0, 40, 2, 16, 1}, {1, 1, 1, 0, 40, 1, 16, 1},                                  // 41..42
};

int default_rows_per_unit(int sched) {
    // one pass per unit: the most wavefronts, which the schedule sweeps favour
    const Schedule& c = kSchedules[sched];
    int U = (64 / c.P) * c.UR;
    if (c.mask && U < 32) U = 32;
    return U > 64 ? 64 : U;
}

namespace {

// Columns per load batch in the tiled kernels: clauses are short, variable
// rows longer.  With one value per lane the registers hold twice the batch:
// the forward then takes 8 columns and schedules may take 16 backward.  A row's last batch takes only
// the columns left, so no batch reads a padding column past the tile's
// length, and the batch length never changes the order of a sum.
constexpr int kChunkF = 4;
constexpr int kChunkB = 8;

// Column count of a load batch, as a type (one instantiation per batch size).
template <int N>
struct Cols {
    static constexpr int value = N;
};

template <int V>
struct VecF {
    float v[V];
};

template <int V>
__device__ __forceinline__ VecF<V> ldv(const float* p) {
    VecF<V> r;
    if constexpr (V == 1) {
        r.v[0] = *p;
    } else if constexpr (V == 2) {
        float2 q = *reinterpret_cast<const float2*>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
    } else {
        float4 q = *reinterpret_cast<const float4*>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
        r.v[2] = q.z;
        r.v[3] = q.w;
    }
    return r;
}

template <int V>
__device__ __forceinline__ void stv(float* p, const VecF<V>& r) {
    if constexpr (V == 1) {
        *p = r.v[0];
    } else if constexpr (V == 2) {
        *reinterpret_cast<float2*>(p) = make_float2(r.v[0], r.v[1]);
    } else {
        *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
    }
}

// OR each aligned group of P ballot bits into its first bit (the row's
// bit is set when any of its P lanes has an unsatisfied restart).
template <int P>
__device__ __forceinline__ uint64_t fold_bits(uint64_t x) {
    if constexpr (P >= 2) x |= x >> 1;
    if constexpr (P >= 4) x |= x >> 2;
    return x;
}

// Compact the ballot bits of lanes 0, P, 2P, ... into consecutive bits.
template <int P>
__device__ __forceinline__ uint64_t compact_bits(uint64_t x) {
    if constexpr (P == 1) {
        return x;
    } else if constexpr (P == 2) {
        x &= 0x5555555555555555ull;
        x = (x | (x >> 1)) & 0x3333333333333333ull;
        x = (x | (x >> 2)) & 0x0f0f0f0f0f0f0f0full;
        x = (x | (x >> 4)) & 0x00ff00ff00ff00ffull;
        x = (x | (x >> 8)) & 0x0000ffff0000ffffull;
        x = (x | (x >> 16)) & 0x00000000ffffffffull;
        return x;
    } else {
        static_assert(P == 4, "bitset schedules use 1, 2 or 4 lanes per row");
        x &= 0x1111111111111111ull;
        x = (x | (x >> 3)) & 0x0303030303030303ull;
        x = (x | (x >> 6)) & 0x000f000f000f000full;
        x = (x | (x >> 12)) & 0x000000ff000000ffull;
        x = (x | (x >> 24)) & 0x000000000000ffffull;
        return x;
    }
}

// ---------------------------------------------------------------------------
// Forward: scores, unsat mask, adjoint a_j = (2/m) mu_j f_j, unit partials.
// Workgroup b works on restart group b % RG; each wave takes a unit of U rows
// of one tile; lane (s, q) handles UR consecutive rows per pass for restarts
// rl..rl+V-1 of the group, column by column so that UR gathers are in flight
// together.  With MASK a row's bit in its restart group's bitset is set when
// the clause is unsatisfied in some restart of the group, and the adjoint is
// written only for rows whose bit is set.
// ---------------------------------------------------------------------------
// `bx` is the workgroup's index within the instance's grid.
template <int P, int V, int UR, bool EVAL, bool MASK>
__device__ __forceinline__ void fwd_body(const FwdArgs& A, const int bx) {
    constexpr int W = 64 / P;
    const int lane = threadIdx.x & 63;
    const int s = lane / P;
    const int q = lane % P;
    if (bx == 0 && threadIdx.x == 0 && A.st != nullptr)
        adam_scalars((double)A.st->t + 1.0, A.lr, A.b1, A.b2, A.st->step_size, A.st->inv_sqrt_bc2);
    const Blocking B = A.B;
    const int rg = bx % B.RG;
    const int tc = __builtin_amdgcn_readfirstlane((bx / B.RG) * 4 + (threadIdx.x >> 6));
    if (tc >= A.ntiles * A.chunks) return;
    const int tile = tc / A.chunks;
    const int chunk = tc % A.chunks;
    const TileDesc d = ldtile(A.tiles + tile);
    const int rl = q * V;
    const int r0 = rg * B.G + rl;
    const bool ract = rl < B.G && r0 < B.R;
    const bool taut = (d.flags & 1u) != 0;
    const float* tg = A.t + (size_t)rg * B.rows_x * B.G;
    float* ag = A.a + (size_t)rg * B.rows_a * B.G;
    const int passes = A.U / (W * UR);
    int64_t cnt[V];
    double los[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        cnt[k] = 0;
        los[k] = 0.0;
    }
    uint64_t mbits = 0;
    for (int pass = 0; pass < passes; ++pass) {
        const int rowin0 = chunk * A.U + pass * (W * UR) + s * UR;
        const uint32_t* e = A.ent + d.base + rowin0;
        // clause weights go out with the entry loads: every row of a tile,
        // padding included, has one, so the load needs no guard
        int64_t wrow[UR];
        if (A.w != nullptr) {
#pragma unroll
            for (int j = 0; j < UR; ++j) wrow[j] = A.w[(size_t)tile * kTile + rowin0 + j];
        }
        float f[UR][V];
        uint32_t allf[UR][V];
#pragma unroll
        for (int j = 0; j < UR; ++j)
#pragma unroll
            for (int k = 0; k < V; ++k) {
                f[j][k] = 0.0f;
                allf[j][k] = ~0u;
            }
        if (ract) {
            if (d.len <= 16) {
                // batches of CF columns, then one batch of the last d.len % CF:
                // all entry loads, then all gathers, then the sums in column
                // order (no padding column is read)
                auto batch = [&](auto nc, const uint32_t c0) {
                    constexpr int NC = decltype(nc)::value;
                    uint32_t en[NC][UR];
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                        for (int j = 0; j < UR; ++j) en[cc][j] = ldc(e + (size_t)(c0 + cc) * kTile + j);
                    VecF<V> tv[NC][UR];
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                        for (int j = 0; j < UR; ++j)
                            tv[cc][j] = ldv<V>(tg + (size_t)(en[cc][j] & kIdx) * B.G + rl);
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                        for (int j = 0; j < UR; ++j)
#pragma unroll
                            for (int k = 0; k < V; ++k) {
                                const uint32_t b = __float_as_uint(tv[cc][j].v[k]) ^ (en[cc][j] & kSign);
                                f[j][k] = f[j][k] + __uint_as_float(b);
                                allf[j][k] &= b;
                            }
                };
                constexpr int CF = V * UR == 1 ? 2 * kChunkF : kChunkF;
                uint32_t c0 = 0;
                for (; c0 + CF <= d.len; c0 += CF) batch(Cols<CF>{}, c0);
                switch (d.len - c0) {
                    case 1: batch(Cols<1>{}, c0); break;
                    case 2: batch(Cols<2>{}, c0); break;
                    case 3: batch(Cols<3>{}, c0); break;
                    case 4: if constexpr (CF > 4) batch(Cols<4>{}, c0); break;
                    case 5: if constexpr (CF > 5) batch(Cols<5>{}, c0); break;
                    case 6: if constexpr (CF > 6) batch(Cols<6>{}, c0); break;
                    case 7: if constexpr (CF > 7) batch(Cols<7>{}, c0); break;
                    default: break;
                }
            } else {
                // long clauses: FP64 accumulation, one row at a time
#pragma unroll
                for (int j = 0; j < UR; ++j) {
                    double fd[V];
#pragma unroll
                    for (int k = 0; k < V; ++k) fd[k] = 0.0;
#pragma unroll 4
                    for (uint32_t c = 0; c < d.len; ++c) {
                        const uint32_t en = ldc(e + (size_t)c * kTile + j);
                        const VecF<V> tv = ldv<V>(tg + (size_t)(en & kIdx) * B.G + rl);
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            const uint32_t b = __float_as_uint(tv.v[k]) ^ (en & kSign);
                            fd[k] = fd[k] + (double)__uint_as_float(b);
                            allf[j][k] &= b;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < V; ++k) f[j][k] = (float)fd[k];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < UR; ++j) {
            const bool real = ract && rowin0 + j < (int)d.nreal;
            // clause weight: a_j = (2/m) mu_j w_j f_j, cost and loss weighted
            // (w = 1 leaves every value bitwise unchanged)
            int64_t wj = 1;
            if (A.w != nullptr && real) wj = wrow[j];
            const float wf = (float)wj;
            VecF<V> av;
            bool any_mu = false;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const bool unsat = real && !taut && (allf[j][k] >> 31) != 0;
                const bool mu = real && (A.all_mode ? true : unsat);
                av.v[k] = mu ? (f[j][k] * wf) * A.two_over_m : 0.0f;
                any_mu = any_mu || mu;
                if (EVAL) {
                    cnt[k] += unsat ? wj : 0;
                    los[k] += mu ? ((double)f[j][k] * (double)f[j][k]) * (double)wj : 0.0;
                }
            }
            if constexpr (MASK) {
                static_assert(UR == 1, "bitset schedules take one row per lane");
                const uint64_t folded = fold_bits<P>(__ballot(any_mu ? 1 : 0));
                mbits |= compact_bits<P>(folded) << (pass * W);
                // every lane of a row whose bit is set writes its restarts
                // (zeros included): the backward pass reads the whole row
                if (ract && ((folded >> (s * P)) & 1u))
                    stv<V>(ag + (size_t)(tile * kTile + rowin0 + j) * B.G + rl, av);
            } else if (ract) {
                stv<V>(ag + (size_t)(tile * kTile + rowin0 + j) * B.G + rl, av);
            }
        }
    }
    if constexpr (MASK) {
        if (lane == 0) {
            uint32_t* w = A.umask + (size_t)rg * A.umask_words + ((size_t)tile * kTile + chunk * A.U) / 32;
            w[0] = (uint32_t)mbits;
            if (A.U == 64) w[1] = (uint32_t)(mbits >> 32);
        }
    }
    if (EVAL) {
#pragma unroll
        for (int off = P; off < 64; off <<= 1) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                cnt[k] += __shfl_xor(cnt[k], off);
                los[k] += __shfl_xor(los[k], off);
            }
        }
        if (s == 0 && ract) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                A.cnt_part[(size_t)tc * B.R + r0 + k] = cnt[k];
                A.loss_part[(size_t)tc * B.R + r0 + k] = los[k];
            }
        }
    }
}

// Index of the instance owning workgroup `b` of a multi-instance launch:
// the last i with b0[i] <= b (b0 is the running sum of the grids).
__device__ __forceinline__ int owner(const int32_t* __restrict__ b0, int32_t n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int P, int V, int UR, bool EVAL, bool MASK>
__global__ __launch_bounds__(256) void k_fwd(FwdArgs A) {
    fwd_body<P, V, UR, EVAL, MASK>(A, blockIdx.x);
}

// Many instances in one launch: instance i owns workgroups [b0[i], b0[i+1]).
template <int P, int V, int UR, bool EVAL, bool MASK>
__global__ __launch_bounds__(256) void k_fwd_multi(const FwdArgs* __restrict__ As, const int32_t* __restrict__ b0,
                                                   int32_t n) {
    const int i = owner(b0, n, blockIdx.x);
    fwd_body<P, V, UR, EVAL, MASK>(As[i], blockIdx.x - b0[i]);
}

// Descriptors of the NT tiles of work unit tc, all loads issued together
// (indexes clamped into the array; tiles past the end get no rows).
template <int NT>
__device__ __forceinline__ void unit_tiles(const TileDesc* tiles, int ntiles, int tc, TileDesc (&d)[NT]) {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int tile = tc * NT + u;
        d[u] = ldtile(tiles + (tile < ntiles ? tile : ntiles - 1));
    }
#pragma unroll
    for (int u = 0; u < NT; ++u)
        if (tc * NT + u >= ntiles) d[u] = TileDesc{0u, 0u, 0u, 0u};
}

// Entry (column c, row `lane`) of a tile, or the padding entry past the row's
// end or when !use.  The load always issues, from a column clamped into the
// tile, so no branch splits a batch of loads.
__device__ __forceinline__ uint32_t unit_entry(const uint32_t* ent, const TileDesc& d, uint32_t c, bool use,
                                               int lane, uint32_t pad) {
    const uint32_t last = d.len > 0 ? d.len - 1 : 0;
    const uint32_t v = ldc(ent + (size_t)d.base + (size_t)(c < last ? c : last) * kTile + lane);
    return use && c < d.len ? v : pad;
}

// ---------------------------------------------------------------------------
// Forward over NT whole tiles per wavefront, one row per lane and one restart
// per row (P = V = 1, 64 rows per tile).  The NT tiles' entry loads, then all
// their gathers, are issued together, so each wavefront keeps NT times the
// reads of the one-tile schedule in flight (it pays where a wavefront's time
// is mostly the wait on its dependent loads: large instances, one restart).
// Work unit u covers tiles [u NT, u NT + NT) and owns one count/loss partial.
// Every row is computed exactly as the one-tile kernel computes it (FP32 sum
// in column order up to 16 columns, FP64 beyond).  MASK = 0 writes every
// row's adjoint; 1 writes the rows in the loss and the tile's unsat bits; 2
// (slot mode) writes the unsat bits and, for the rows in the loss now or one
// step ago, the signed adjoint (or 0) into each occurrence's variable-side slot.
// ---------------------------------------------------------------------------
template <int NT, bool EVAL, int MASK>
__device__ __forceinline__ void fwd_nt_body(const FwdArgs& A, const int bx) {
    const int lane = threadIdx.x & 63;
    if (bx == 0 && threadIdx.x == 0 && A.st != nullptr)
        adam_scalars((double)A.st->t + 1.0, A.lr, A.b1, A.b2, A.st->step_size, A.st->inv_sqrt_bc2);
    const Blocking B = A.B;  // G = 1: restart group rg is restart rg
    const int rg = bx % B.RG;
    const int tc = __builtin_amdgcn_readfirstlane((bx / B.RG) * 4 + (threadIdx.x >> 6));
    if (tc >= (A.ntiles + NT - 1) / NT) return;
    const float* tg = A.t + (size_t)rg * B.rows_x;
    float* ag = A.a + (size_t)rg * B.rows_a;
    TileDesc d[NT];
    unit_tiles<NT>(A.tiles, A.ntiles, tc, d);
    uint32_t lmax = 0;  // longest short (<= 16 column) tile of the unit
#pragma unroll
    for (int u = 0; u < NT; ++u)
        if (d[u].len <= 16) lmax = d[u].len > lmax ? d[u].len : lmax;
    // clause weights go out before the gathers (rows of tiles past the end
    // read tile 0's, unused)
    int64_t wrow[NT];
    if (A.w != nullptr) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int tile = tc * NT + u;
            wrow[u] = A.w[(size_t)(tile < A.ntiles ? tile : 0) * kTile + lane];
        }
    }
    float f[NT];
    uint32_t allf[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        f[u] = 0.0f;
        allf[u] = ~0u;
    }
    // batches of CF columns, then one batch of the last lmax % CF
    auto batch = [&](auto nc, const uint32_t c0) {
        constexpr int NC = decltype(nc)::value;
        uint32_t en[NC][NT];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
#pragma unroll
            for (int u = 0; u < NT; ++u)
                en[cc][u] = unit_entry(A.ent, d[u], c0 + cc, d[u].len <= 16, lane, A.pad_entry);
        float tv[NC][NT];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
#pragma unroll
            for (int u = 0; u < NT; ++u) tv[cc][u] = tg[en[cc][u] & kIdx];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const uint32_t b = __float_as_uint(tv[cc][u]) ^ (en[cc][u] & kSign);
                f[u] = f[u] + __uint_as_float(b);
                allf[u] &= b;
            }
    };
    constexpr int CF = 2 * kChunkF;  // one value per lane
    uint32_t c0 = 0;
    for (; c0 + CF <= lmax; c0 += CF) batch(Cols<CF>{}, c0);
    switch (lmax - c0) {
        case 1: batch(Cols<1>{}, c0); break;
        case 2: batch(Cols<2>{}, c0); break;
        case 3: batch(Cols<3>{}, c0); break;
        case 4: batch(Cols<4>{}, c0); break;
        case 5: batch(Cols<5>{}, c0); break;
        case 6: batch(Cols<6>{}, c0); break;
        case 7: batch(Cols<7>{}, c0); break;
        default: break;
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        if (d[u].len <= 16) continue;
        // long clauses: FP64 accumulation, as in the one-tile kernel
        double fd = 0.0;
        for (uint32_t c = 0; c < d[u].len; ++c) {
            const uint32_t en = ldc(A.ent + d[u].base + (size_t)c * kTile + lane);
            const uint32_t b = __float_as_uint(tg[en & kIdx]) ^ (en & kSign);
            fd = fd + (double)__uint_as_float(b);
            allf[u] &= b;
        }
        f[u] = (float)fd;
    }
    int64_t cnt = 0;
    double los = 0.0;
    bool put[NT];       // slot mode: row's occurrences get a value this step
    uint32_t pval[NT];  // slot mode: the row's adjoint bits (0 outside the loss)
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        put[u] = false;
        pval[u] = 0u;
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int tile = tc * NT + u;
        if (tile >= A.ntiles) break;
        const bool real = lane < (int)d[u].nreal;
        const bool taut = (d[u].flags & 1u) != 0;
        const size_t row = (size_t)tile * kTile + lane;
        int64_t wj = 1;
        if (A.w != nullptr && real) wj = wrow[u];
        const float wf = (float)wj;
        const bool unsat = real && !taut && (allf[u] >> 31) != 0;
        const bool mu = real && (A.all_mode ? true : unsat);
        const float av = mu ? (f[u] * wf) * A.two_over_m : 0.0f;
        if (EVAL) {
            cnt += unsat ? wj : 0;
            los += mu ? ((double)f[u] * (double)f[u]) * (double)wj : 0.0;
        }
        if constexpr (MASK == 1) {
            const uint64_t bits = __ballot(mu ? 1 : 0);
            if (mu) ag[row] = av;
            if (lane == 0) {
                uint32_t* w = A.umask + (size_t)rg * A.umask_words + (size_t)tile * 2;
                w[0] = (uint32_t)bits;
                w[1] = (uint32_t)(bits >> 32);
            }
        } else if constexpr (MASK == 2) {
            // the tile's bits of the step before say which rows still hold
            // their adjoint in the occurrence slots; this step's replace them
            const uint64_t bits = __ballot(mu ? 1 : 0);
            uint32_t* w = A.umask + (size_t)rg * A.umask_words + (size_t)tile * 2;
            const uint64_t was = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
            put[u] = mu || ((was >> lane) & 1u) != 0;
            pval[u] = __float_as_uint(av);
            if (lane == 0) {
                w[0] = (uint32_t)bits;
                w[1] = (uint32_t)(bits >> 32);
            }
        } else {
            ag[row] = av;
        }
    }
    if constexpr (MASK == 2) {
        // every occurrence of a row in the loss, or that was in it one step
        // ago, gets the row's adjoint (signed by its literal) or 0 in its
        // variable-side slot; slots of other rows already hold 0.  The slot
        // loads of a batch go out together.  A tile's slots are stored row by
        // row, so the few rows that need theirs fetch few lines.
        uint32_t smax = 0;
#pragma unroll
        for (int u = 0; u < NT; ++u)
            if (__ballot(put[u] ? 1 : 0) != 0) smax = d[u].len > smax ? d[u].len : smax;
        for (uint32_t c0 = 0; c0 < smax; c0 += 8) {
            uint32_t sl[8][NT];
#pragma unroll
            for (int cc = 0; cc < 8; ++cc)
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    sl[cc][u] = (put[u] && c0 + cc < d[u].len)
                                    ? A.slot[(size_t)d[u].base + (size_t)lane * d[u].len + c0 + cc]
                                    : kNoSlot;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc)
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    if (sl[cc][u] != kNoSlot) A.contrib[sl[cc][u] & kIdx] = __uint_as_float(pval[u] ^ (sl[cc][u] & kSign));
        }
    }
    if (EVAL) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            cnt += __shfl_xor(cnt, off);
            los += __shfl_xor(los, off);
        }
        if (lane == 0) {
            A.cnt_part[(size_t)tc * B.R + rg] = cnt;
            A.loss_part[(size_t)tc * B.R + rg] = los;
        }
    }
}

template <int NT, bool EVAL, int MASK>
__global__ __launch_bounds__(256) void k_fwd_nt(FwdArgs A) {
    fwd_nt_body<NT, EVAL, MASK>(A, blockIdx.x);
}

template <int NT, bool EVAL, int MASK>
__global__ __launch_bounds__(256) void k_fwd_nt_multi(const FwdArgs* __restrict__ As,
                                                      const int32_t* __restrict__ b0, int32_t n) {
    const int i = owner(b0, n, blockIdx.x);
    fwd_nt_body<NT, EVAL, MASK>(As[i], blockIdx.x - b0[i]);
}

// ---------------------------------------------------------------------------
// Epilogue of a variable: g = sech^2(x) G, then the optimizer step (or the
// gradient itself), t = signed tanh of the new x.  `base` is the element
// offset of (variable, first restart) in the blocked state arrays; r0 is the
// first restart's index.
// ---------------------------------------------------------------------------
template <int V, int OPT>
struct VarState {
    VecF<V> x, m, v;
};

// Loads of the epilogue's inputs, issued before the transposed sum so they
// overlap its gathers.
template <int V, int OPT>
__device__ __forceinline__ VarState<V, OPT> var_load(const BwdArgs& A, size_t base) {
    VarState<V, OPT> st;
    st.x = ldv<V>(A.x + base);
    if constexpr (OPT == kAdam) {
        st.m = ldv<V>(A.m + base);
        st.v = ldv<V>(A.v + base);
    }
    return st;
}

template <int V, int OPT>
__device__ __forceinline__ void var_epilogue(const BwdArgs& A, size_t base, int r0, const double (&G)[V],
                                             VarState<V, OPT> st) {
    VecF<V>& xv = st.x;
    if (A.eval) {
#pragma unroll
        for (int k = 0; k < V; ++k)
            if (A.improved[r0 + k]) A.best_a[base + k] = xv.v[k] > 0.0f ? 1 : 0;
    }
    float g[V];
#pragma unroll
    for (int k = 0; k < V; ++k) g[k] = grad_of(xv.v[k], G[k]);
    if constexpr (OPT == kGrad) {
        VecF<V> gv;
#pragma unroll
        for (int k = 0; k < V; ++k) gv.v[k] = g[k];
        stv<V>(A.g_out + base, gv);
        return;
    } else if constexpr (OPT == kSgd) {
        VecF<V> tv;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            xv.v[k] = xv.v[k] - A.lr * g[k];
            tv.v[k] = signed_tanh(xv.v[k]);
        }
        stv<V>(A.x + base, xv);
        stv<V>(A.t + base, tv);
    } else {
        const float ss = A.st->step_size;
        const float ib2 = A.st->inv_sqrt_bc2;
        const AdamCoef co{A.b1, A.b2, A.eps, A.omb1, A.omb2};
        VecF<V>& mv = st.m;
        VecF<V>& vv = st.v;
        VecF<V> tv;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            adam_update(xv.v[k], mv.v[k], vv.v[k], g[k], ss, ib2, co);
            tv.v[k] = signed_tanh(xv.v[k]);
        }
        stv<V>(A.m + base, mv);
        stv<V>(A.v + base, vv);
        stv<V>(A.x + base, xv);
        stv<V>(A.t + base, tv);
    }
}

template <int V, int OPT>
__device__ __forceinline__ void var_epilogue(const BwdArgs& A, size_t base, int r0, const double (&G)[V]) {
    var_epilogue<V, OPT>(A, base, r0, G, var_load<V, OPT>(A, base));
}

// ---------------------------------------------------------------------------
// Backward: transposed sums G = sum_j W_ij a_j over variable rows (atomic-free;
// each (row, restart) summed by one lane in FP64 in entry order), fused
// epilogue for whole rows, partials for heavy-row segments.  MASK = 0 gathers
// every entry's clause adjoint; 1 gathers it only when the clause's unsat bit
// is set (it is 0 otherwise); 2 (slot mode) reads the occurrence slots that
// the forward filled, parallel to the entries, with no index load or gather.
// ---------------------------------------------------------------------------
template <int P, int V, int UR, int OPT, int MASK, int CB>
__device__ __forceinline__ void bwd_body(const BwdArgs& A, const int bx) {
    static_assert(CB == kChunkB || (CB == 2 * kChunkB && V * UR == 1), "long batches take one value per lane");
    static_assert(MASK != 2 || (P == 1 && V == 1 && UR == 1), "slot mode takes one restart and one row per lane");
    constexpr int W = 64 / P;
    const int lane = threadIdx.x & 63;
    const int s = lane / P;
    const int q = lane % P;
    if (OPT != kGrad && bx == 0 && threadIdx.x == 0) A.st->t += 1;
    const Blocking B = A.B;
    const int rg = bx % B.RG;
    const int tc = __builtin_amdgcn_readfirstlane((bx / B.RG) * 4 + (threadIdx.x >> 6));
    if (tc >= A.ntiles * A.chunks) return;
    const int tile = tc / A.chunks;
    const int chunk = tc % A.chunks;
    const TileDesc d = ldtile(A.tiles + tile);
    const int rl = q * V;
    const int r0 = rg * B.G + rl;
    if (rl >= B.G || r0 >= B.R) return;
    const bool segtile = tile < A.seg_tiles;
    const float* ag = A.a + (size_t)rg * B.rows_a * B.G;
    const uint32_t* um = A.umask + (size_t)rg * A.umask_words;
    const size_t xbase = (size_t)rg * B.rows_x * B.G;
    double* sg = A.seg_part + (size_t)rg * B.rows_seg * B.G;
    const int passes = A.U / (W * UR);
    for (int pass = 0; pass < passes; ++pass) {
        const int rowin0 = chunk * A.U + pass * (W * UR) + s * UR;
        if (rowin0 >= (int)d.nreal) break;
        const uint32_t* e = A.ent + d.base + rowin0;
        const float* cs = MASK == 2 ? A.contrib + d.base + rowin0 : nullptr;
        double G[UR][V];
#pragma unroll
        for (int j = 0; j < UR; ++j)
#pragma unroll
            for (int k = 0; k < V; ++k) G[j][k] = 0.0;
        // with one value per lane the epilogue's x, m, v loads go out before
        // the transposed sums, so they wait alongside the gathers (wider
        // schedules would lose a wave per SIMD to the registers)
        constexpr bool kEarly = V * UR == 1;
        VarState<V, OPT> st[UR];
        if (kEarly && !segtile) {
#pragma unroll
            for (int j = 0; j < UR; ++j)
                if (rowin0 + j < (int)d.nreal)
                    st[j] = var_load<V, OPT>(
                        A, xbase + (size_t)(A.n_heavy + (tile * kTile + rowin0 + j - A.seg_tiles * kTile)) * B.G + rl);
        }
        // batches of CB columns, then one batch of the last d.len % CB: all
        // entry loads, then all gathers, then the sums in column order (no
        // padding column is read)
        auto batch = [&](auto nc, const uint32_t c0) {
            constexpr int NC = decltype(nc)::value;
            if constexpr (MASK == 2) {
                // slot mode: the forward left each occurrence's signed
                // adjoint (or 0) in the slot parallel to its entry
                float cv[NC];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) cv[cc] = cs[(size_t)(c0 + cc) * kTile];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) G[0][0] = G[0][0] + (double)cv[cc];
                return;
            }
            uint32_t en[NC][UR];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                for (int j = 0; j < UR; ++j) en[cc][j] = ldc(e + (size_t)(c0 + cc) * kTile + j);
            VecF<V> av[NC][UR];
            if constexpr (MASK == 1) {
                uint32_t w[NC][UR];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                    for (int j = 0; j < UR; ++j) w[cc][j] = um[(en[cc][j] & kIdx) >> 5];
                // a satisfied clause's adjoint is 0: read the always-zero row
                // instead (one cached line), so every gather issues at once
#pragma unroll
                for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                    for (int j = 0; j < UR; ++j) {
                        const uint32_t row = en[cc][j] & kIdx;
                        const uint32_t src = ((w[cc][j] >> (row & 31)) & 1u) ? row : (A.pad_entry & kIdx);
                        av[cc][j] = ldv<V>(ag + (size_t)src * B.G + rl);
                    }
            } else {
#pragma unroll
                for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                    for (int j = 0; j < UR; ++j)
                        av[cc][j] = ldv<V>(ag + (size_t)(en[cc][j] & kIdx) * B.G + rl);
            }
#pragma unroll
            for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                for (int j = 0; j < UR; ++j)
#pragma unroll
                    for (int k = 0; k < V; ++k)
                        G[j][k] = G[j][k] + (double)__uint_as_float(__float_as_uint(av[cc][j].v[k]) ^ (en[cc][j] & kSign));
        };
        uint32_t c0 = 0;
        for (; c0 + CB <= d.len; c0 += CB) batch(Cols<CB>{}, c0);
        static_assert(CB <= 16, "one case per remainder");
        switch (d.len - c0) {
            case 1: if constexpr (CB > 1) batch(Cols<1>{}, c0); break;
            case 2: if constexpr (CB > 2) batch(Cols<2>{}, c0); break;
            case 3: if constexpr (CB > 3) batch(Cols<3>{}, c0); break;
            case 4: if constexpr (CB > 4) batch(Cols<4>{}, c0); break;
            case 5: if constexpr (CB > 5) batch(Cols<5>{}, c0); break;
            case 6: if constexpr (CB > 6) batch(Cols<6>{}, c0); break;
            case 7: if constexpr (CB > 7) batch(Cols<7>{}, c0); break;
            case 8: if constexpr (CB > 8) batch(Cols<8>{}, c0); break;
            case 9: if constexpr (CB > 9) batch(Cols<9>{}, c0); break;
            case 10: if constexpr (CB > 10) batch(Cols<10>{}, c0); break;
            case 11: if constexpr (CB > 11) batch(Cols<11>{}, c0); break;
            case 12: if constexpr (CB > 12) batch(Cols<12>{}, c0); break;
            case 13: if constexpr (CB > 13) batch(Cols<13>{}, c0); break;
            case 14: if constexpr (CB > 14) batch(Cols<14>{}, c0); break;
            case 15: if constexpr (CB > 15) batch(Cols<15>{}, c0); break;
            default: break;
        }
#pragma unroll
        for (int j = 0; j < UR; ++j) {
            if (rowin0 + j >= (int)d.nreal) break;
            const int row = tile * kTile + rowin0 + j;
            if (segtile) {
#pragma unroll
                for (int k = 0; k < V; ++k) sg[(size_t)row * B.G + rl + k] = G[j][k];
            } else {
                const int var = A.n_heavy + (row - A.seg_tiles * kTile);
                if constexpr (kEarly)
                    var_epilogue<V, OPT>(A, xbase + (size_t)var * B.G + rl, r0, G[j], st[j]);
                else
                    var_epilogue<V, OPT>(A, xbase + (size_t)var * B.G + rl, r0, G[j]);
            }
        }
    }
}

template <int P, int V, int UR, int OPT, int MASK, int CB = kChunkB>
__global__ __launch_bounds__(256) void k_bwd(BwdArgs A) {
    bwd_body<P, V, UR, OPT, MASK, CB>(A, blockIdx.x);
}

template <int P, int V, int UR, int OPT, int MASK, int CB = kChunkB>
__global__ __launch_bounds__(256) void k_bwd_multi(const BwdArgs* __restrict__ As, const int32_t* __restrict__ b0,
                                                   int32_t n) {
    const int i = owner(b0, n, blockIdx.x);
    bwd_body<P, V, UR, OPT, MASK, CB>(As[i], blockIdx.x - b0[i]);
}

// Heavy variables: combine segment partials in a fixed order that depends on
// the instance only.  A variable with at most kWideSegs segments uses 64
// slots (one wavefront): slot q sums segments q, q+64, ... in order, then a
// fixed halving tree.  Wider variables use 1024 slots (one workgroup) the same
// way.  One launch of 1024-thread workgroups: the first n_heavy_wide * R
// workgroups take one wide (variable, restart) each, the rest take sixteen
// narrow ones (one per wavefront).
//
// The kernel moves little data and is bound by its chain of dependent loads,
// so the epilogue's inputs are loaded before the sums, a slot's partials load
// NB at a time (a wide slot has at most ~13, so one batch) with the address of
// a slot past the end clamped to a valid one and its value not added, and the
// last six levels of the wide tree run as wavefront shuffles (the pairing is
// the same as in LDS).
template <int NB>
__device__ __forceinline__ double slot_sum(const double* __restrict__ sg, const int G, const int q0, const int p1,
                                           const int stride) {
    double u = 0.0;
    for (int q = q0; q < p1; q += stride * NB) {
        double val[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) val[k] = sg[(size_t)min(q + k * stride, p1 - 1) * G];
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (q + k * stride < p1) u = u + val[k];
    }
    return u;
}

template <int OPT>
__device__ __forceinline__ void combine_body(const BwdArgs& A, const int bx, double* su) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const Blocking B = A.B;
    const int nwide = A.n_heavy_wide * B.R;
    int h, r;
    if (bx < nwide) {
        h = bx / B.R;
        r = bx % B.R;
    } else {
        const int w = (bx - nwide) * 16 + (tid >> 6);
        if (w >= (A.n_heavy - A.n_heavy_wide) * B.R) return;
        h = A.n_heavy_wide + w / B.R;
        r = w % B.R;
    }
    const size_t base = ((size_t)(r / B.G) * B.rows_x + h) * B.G + r % B.G;
    const VarState<1, OPT> st = var_load<1, OPT>(A, base);
    const double* sg = A.seg_part + (size_t)(r / B.G) * B.rows_seg * B.G + r % B.G;
    const int p0 = A.seg_first[h];
    const int p1 = A.seg_first[h + 1];
    double u;
    if (bx < nwide) {
        u = slot_sum<8>(sg, B.G, p0 + tid, p1, 1024);
        su[tid] = u;
        __syncthreads();
        for (int s = 512; s >= 64; s >>= 1) {
            if (tid < s) su[tid] = su[tid] + su[tid + s];
            __syncthreads();
        }
        if (tid >= 64) return;
        u = su[tid];
    } else {
        u = slot_sum<4>(sg, B.G, p0 + lane, p1, 64);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) u = u + __shfl_down(u, off);
    if (lane != 0) return;
    double G[1] = {u};
    var_epilogue<1, OPT>(A, base, r, G, st);
}

template <int OPT>
__global__ __launch_bounds__(1024) void k_combine(BwdArgs A) {
    __shared__ double su[1024];
    combine_body<OPT>(A, blockIdx.x, su);
}

template <int OPT>
__global__ __launch_bounds__(1024) void k_combine_multi(const BwdArgs* __restrict__ As,
                                                        const int32_t* __restrict__ b0, int32_t n) {
    __shared__ double su[1024];
    const int i = owner(b0, n, blockIdx.x);
    combine_body<OPT>(As[i], blockIdx.x - b0[i], su);
}

// Count/loss partials are summed in two fixed stages.  Stage 1: block
// (restart block rb, chunk c) sums units [c * CH, (c + 1) * CH) for 64
// restarts: lane l of the 256 threads holds restart 64 rb + (l % RP) and slot
// l / RP; a slot sums its units with stride NS = 256 / RP in order, then a
// fixed tree over the slots.  Stage 2 sums the chunk partials the same way
// with one 1024-thread block per restart block, and tracks the best.  When
// the unit partials are few (n_chunks == 0), stage 2 sums them directly and
// stage 1 is not launched.
__device__ __forceinline__ int restart_lanes(int R) {
    int RP = 1;  // restarts side by side: the next power of two >= R, at most 64
    while (RP < 64 && RP < R) RP <<= 1;
    return RP;
}

__device__ __forceinline__ void reduce1_body(const ReduceArgs& A, const int bx, const int by, int64_t* sc,
                                             double* sl) {
    const int tid = threadIdx.x;
    const int RP = restart_lanes(A.R);
    const int NS = 256 / RP;
    const int rloc = tid % RP;
    const int slot = tid / RP;
    const int r = bx * 64 + rloc;
    const int u0 = by * A.chunk;
    const int u1 = min(u0 + A.chunk, A.n_units);
    int64_t c = 0;
    double l = 0.0;
    if (r < A.R) {
#pragma unroll 8
        for (int u = u0 + slot; u < u1; u += NS) {
            c += A.cnt_part[(size_t)u * A.R + r];
            l = l + A.loss_part[(size_t)u * A.R + r];
        }
    }
    sc[tid] = c;
    sl[tid] = l;
    __syncthreads();
    for (int h = NS / 2; h >= 1; h >>= 1) {
        if (slot < h) {
            sc[tid] += sc[tid + h * RP];
            sl[tid] = sl[tid] + sl[tid + h * RP];
        }
        __syncthreads();
    }
    if (slot == 0 && r < A.R) {
        A.cnt_mid[(size_t)by * A.R + r] = sc[tid];
        A.loss_mid[(size_t)by * A.R + r] = sl[tid];
    }
}

__global__ __launch_bounds__(256) void k_reduce1(ReduceArgs A) {
    __shared__ int64_t sc[256];
    __shared__ double sl[256];
    reduce1_body(A, blockIdx.x, blockIdx.y, sc, sl);
}

// Multi-instance stage 1: instance i's grid is ceil(R/64) x n_chunks, flattened.
__global__ __launch_bounds__(256) void k_reduce1_multi(const ReduceArgs* __restrict__ As,
                                                       const int32_t* __restrict__ b0, int32_t n) {
    __shared__ int64_t sc[256];
    __shared__ double sl[256];
    const int i = owner(b0, n, blockIdx.x);
    const ReduceArgs& A = As[i];
    const int gx = (A.R + 63) / 64;
    const int lb = blockIdx.x - b0[i];
    reduce1_body(A, lb % gx, lb / gx, sc, sl);
}

__device__ __forceinline__ void reduce2_body(const ReduceArgs& A, const int bx, int64_t* sc, double* sl) {
    const int tid = threadIdx.x;
    const int RP = restart_lanes(A.R);
    const int NS = 1024 / RP;
    const int rloc = tid % RP;
    const int slot = tid / RP;
    const int r = bx * 64 + rloc;
    int64_t c = 0;
    double l = 0.0;
    // with no stage-1 chunks the unit partials are few enough to sum here
    const bool direct = A.n_chunks == 0;
    const int nsrc = direct ? A.n_units : A.n_chunks;
    const int64_t* __restrict__ cp = direct ? A.cnt_part : A.cnt_mid;
    const double* __restrict__ lp = direct ? A.loss_part : A.loss_mid;
    if (r < A.R) {
#pragma unroll 8
        for (int u = slot; u < nsrc; u += NS) {
            c += cp[(size_t)u * A.R + r];
            l = l + lp[(size_t)u * A.R + r];
        }
    }
    sc[tid] = c;
    sl[tid] = l;
    __syncthreads();
    for (int h = NS / 2; h >= 1; h >>= 1) {
        if (slot < h) {
            sc[tid] += sc[tid + h * RP];
            sl[tid] = sl[tid] + sl[tid + h * RP];
        }
        __syncthreads();
    }
    if (slot == 0 && r < A.R) {
        const int64_t count = sc[tid] + A.n_empty;
        A.cur_count[r] = count;
        A.cur_loss[r] = sl[tid] * A.inv_m;
        if (A.trace != nullptr) {
            const int32_t t = A.st->t;
            const int32_t row = (int32_t)((((int64_t)t + A.trace_k - 1) / A.trace_k - A.trace_base) % A.trace_cap);
            A.trace[(size_t)row * A.R + r] = TracePoint{t, 0, count, sl[tid] * A.inv_m};
        }
        if (A.track) {
            if (count < A.best[r]) {
                A.best[r] = count;
                A.best_step[r] = A.st->t;
                A.improved[r] = 1;
            } else {
                A.improved[r] = 0;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_reduce(ReduceArgs A) {
    __shared__ int64_t sc[1024];
    __shared__ double sl[1024];
    reduce2_body(A, blockIdx.x, sc, sl);
}

// Multi-instance stage 2: instance i's grid is ceil(R/64).
__global__ __launch_bounds__(1024) void k_reduce_multi(const ReduceArgs* __restrict__ As,
                                                       const int32_t* __restrict__ b0, int32_t n) {
    __shared__ int64_t sc[1024];
    __shared__ double sl[1024];
    const int i = owner(b0, n, blockIdx.x);
    reduce2_body(As[i], blockIdx.x - b0[i], sc, sl);
}

// Element offset of (row, restart r) in a blocked array with `rows` rows.
__device__ __forceinline__ size_t boff(const Blocking& B, int rows, int row, int r) {
    return ((size_t)(r / B.G) * rows + row) * B.G + (r % B.G);
}

// State initialisation: x^0 (caller values, an assignment, or SplitMix64),
// t = signed tanh(x), zero moments, the dummy rows, best = m.
__global__ __launch_bounds__(256) void k_init(InitArgs A) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const Blocking B = A.B;
    const int64_t total = (int64_t)A.n * B.R;
    if (idx < total) {
        const int32_t i = (int32_t)(idx / B.R);
        const int32_t r = (int32_t)(idx % B.R);
        const int32_t o = A.var_old[i];
        float x;
        if (A.x0 != nullptr) {
            x = A.x0[(size_t)o * B.R + r];
        } else if (A.assign0 != nullptr) {
            x = A.assign0[o] ? 1.0f : -1.0f;
        } else {
            const uint64_t z = splitmix64(A.seed + (uint64_t)r, (uint64_t)o + 1);
            x = 2.0f * ((float)(z >> 40) * (1.0f / 16777216.0f)) - 1.0f;
        }
        const size_t e = boff(B, B.rows_x, i, r);
        A.x[e] = x;
        A.t[e] = signed_tanh(x);
        if (A.mm != nullptr) {
            A.mm[e] = A.m0 != nullptr ? A.m0[(size_t)o * B.R + r] : 0.0f;
            A.vv[e] = A.v0 != nullptr ? A.v0[(size_t)o * B.R + r] : 0.0f;
        }
        if (A.best_a != nullptr)
            A.best_a[e] = A.best_a0 != nullptr ? (A.best_a0[(size_t)r * A.n + o] != 0 ? 1 : 0) : (x > 0.0f ? 1 : 0);
    }
    if (idx < B.R) {
        const int r = (int)idx;
        A.t[boff(B, B.rows_x, A.n, r)] = -0.0f;
        if (A.a != nullptr) A.a[boff(B, B.rows_a, A.a_zero_row, r)] = 0.0f;
        if (A.best != nullptr) {
            if (!A.keep_best) {
                A.best[r] = A.best0;
                A.best_step[r] = -1;
            }
            A.improved[r] = 0;
        }
    }
    if (A.umask != nullptr && idx < A.umask_words) A.umask[idx] = 0u;
    if (A.contrib != nullptr && idx < A.contrib_n) A.contrib[idx] = 0.0f;
    if (idx == 0 && A.st != nullptr) {
        A.st->t = A.step0;
        A.st->step_size = 0.0f;
        A.st->inv_sqrt_bc2 = 1.0f;
    }
}

__global__ __launch_bounds__(256) void k_slot_fill(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = kNoSlot;
}

// One thread per variable-side row: for each of the row's entries, the entry
// of its clause row that holds the row's variable (each variable appears at
// most once in a canonical clause) gets this entry's index and sign.
__global__ __launch_bounds__(256) void k_slots(SlotArgs A) {
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (int64_t)A.v_tiles * kTile) return;
    const int32_t tile = (int32_t)(gid / kTile), q = (int32_t)(gid % kTile);
    const TileDesc d = A.v_tile[tile];
    if (q >= (int32_t)d.nreal) return;
    const int32_t row = tile * kTile + q;
    int32_t v;
    if (row < A.seg_rows) {
        // the heavy variable whose segments hold this row: the last h with
        // seg_first[h] <= row
        int32_t lo = 0, hi = A.n_heavy;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) / 2;
            if (A.seg_first[mid] <= row) lo = mid; else hi = mid;
        }
        v = lo;
    } else {
        v = A.n_heavy + (row - A.seg_tiles * kTile);
    }
    for (uint32_t c = 0; c < d.len; ++c) {
        const uint32_t vpos = d.base + c * kTile + (uint32_t)q;
        const uint32_t e = A.v_ent[vpos];
        if (e == A.vpad) continue;
        const uint32_t j = e & kIdx;
        const TileDesc cd = A.c_tile[j / kTile];
        for (uint32_t cc = 0; cc < cd.len; ++cc) {
            const uint32_t cpos = cd.base + cc * kTile + j % kTile;
            if ((A.c_ent[cpos] & kIdx) == (uint32_t)v) {
                A.c_slot[cd.base + (j % kTile) * cd.len + cc] = vpos | (e & kSign);  // row-major in the tile
                break;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_snapshot(int32_t n_act, Blocking B, const float* x,
                                                   const int32_t* improved, uint8_t* best_a) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n_act * B.R) return;
    const int32_t i = (int32_t)(idx / B.R);
    const int32_t r = (int32_t)(idx % B.R);
    if (improved[r]) {
        const size_t e = boff(B, B.rows_x, i, r);
        best_a[e] = x[e] > 0.0f ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_extract(int32_t n, Blocking B, int32_t r, const int32_t* var_old,
                                                  const uint8_t* best_a, uint8_t* out) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    out[var_old[i]] = best_a[boff(B, B.rows_x, i, r)];
}

__global__ __launch_bounds__(256) void k_scatter_bytes(int32_t n, Blocking B, const int32_t* var_old,
                                                       const uint8_t* src, uint8_t* dst) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * B.R) return;
    const int32_t i = (int32_t)(idx / B.R);
    const int32_t r = (int32_t)(idx % B.R);
    dst[(size_t)r * n + var_old[i]] = src[boff(B, B.rows_x, i, r)];
}

__global__ __launch_bounds__(256) void k_scatter(int32_t n, int32_t n_act, Blocking B, const int32_t* var_old,
                                                  const float* src, float* dst, const float* scale) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * B.R) return;
    const int32_t i = (int32_t)(idx / B.R);
    const int32_t r = (int32_t)(idx % B.R);
    float v = i < n_act ? src[boff(B, B.rows_x, i, r)] : 0.0f;
    if (scale != nullptr) v = scale[r] * v;
    dst[(size_t)var_old[i] * B.R + r] = v;
}

template <int P, int V, int UR, int MASK, int CB = kChunkB>
hipError_t fwd_for(bool eval, const FwdArgs& A, int blocks, hipStream_t s) {
    if (eval)
        hipLaunchKernelGGL((k_fwd<P, V, UR, true, MASK != 0>), dim3(blocks), dim3(256), 0, s, A);
    else
        hipLaunchKernelGGL((k_fwd<P, V, UR, false, MASK != 0>), dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

template <int P, int V, int UR, int MASK, int CB = kChunkB>
hipError_t fwd_multi_for(bool eval, const MultiLaunch& M, hipStream_t s) {
    if (eval)
        hipLaunchKernelGGL((k_fwd_multi<P, V, UR, true, MASK != 0>), dim3(M.blocks), dim3(256), 0, s,
                           static_cast<const FwdArgs*>(M.args), M.b0, M.n);
    else
        hipLaunchKernelGGL((k_fwd_multi<P, V, UR, false, MASK != 0>), dim3(M.blocks), dim3(256), 0, s,
                           static_cast<const FwdArgs*>(M.args), M.b0, M.n);
    return hipGetLastError();
}

template <int P, int V, int UR, int MASK, int CB = kChunkB>
hipError_t bwd_multi_for(int opt, const MultiLaunch& M, hipStream_t s) {
    const BwdArgs* a = static_cast<const BwdArgs*>(M.args);
    if (opt == kAdam)
        hipLaunchKernelGGL((k_bwd_multi<P, V, UR, kAdam, MASK, CB>), dim3(M.blocks), dim3(256), 0, s, a, M.b0,
                           M.n);
    else
        hipLaunchKernelGGL((k_bwd_multi<P, V, UR, kSgd, MASK, CB>), dim3(M.blocks), dim3(256), 0, s, a, M.b0,
                           M.n);
    return hipGetLastError();
}

template <int NT, int MASK, int CB = kChunkB>
hipError_t fwd_for_nt(bool eval, const FwdArgs& A, int blocks, hipStream_t s) {
    if (eval)
        hipLaunchKernelGGL((k_fwd_nt<NT, true, MASK>), dim3(blocks), dim3(256), 0, s, A);
    else
        hipLaunchKernelGGL((k_fwd_nt<NT, false, MASK>), dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

template <int NT, int MASK, int CB = kChunkB>
hipError_t fwd_multi_for_nt(bool eval, const MultiLaunch& M, hipStream_t s) {
    const FwdArgs* a = static_cast<const FwdArgs*>(M.args);
    if (eval)
        hipLaunchKernelGGL((k_fwd_nt_multi<NT, true, MASK>), dim3(M.blocks), dim3(256), 0, s, a, M.b0, M.n);
    else
        hipLaunchKernelGGL((k_fwd_nt_multi<NT, false, MASK>), dim3(M.blocks), dim3(256), 0, s, a, M.b0, M.n);
    return hipGetLastError();
}

template <int P, int V, int UR, int MASK, int CB = kChunkB>
hipError_t bwd_for(int opt, const BwdArgs& A, int blocks, hipStream_t s) {
    if (opt == kAdam)
        hipLaunchKernelGGL((k_bwd<P, V, UR, kAdam, MASK, CB>), dim3(blocks), dim3(256), 0, s, A);
    else if (opt == kSgd)
        hipLaunchKernelGGL((k_bwd<P, V, UR, kSgd, MASK, CB>), dim3(blocks), dim3(256), 0, s, A);
    else
        hipLaunchKernelGGL((k_bwd<P, V, UR, kGrad, MASK, CB>), dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

// The multi-tile entries differ in the forward only: their backward is the
// one-row-per-lane kernel.
template <int NT, int MASK, int CB = kChunkB>
hipError_t bwd_for_nt(int opt, const BwdArgs& A, int blocks, hipStream_t s) {
    return bwd_for<1, 1, 1, MASK, CB>(opt, A, blocks, s);
}

template <int NT, int MASK, int CB = kChunkB>
hipError_t bwd_multi_for_nt(int opt, const MultiLaunch& M, hipStream_t s) {
    return bwd_multi_for<1, 1, 1, MASK, CB>(opt, M, s);
}

}  // namespace

#define HMS_SCHED_SWITCH(FN, ...)                          \
    switch (sched) {                                       \
        case 1: return FN<1, 1, 1, 0>(__VA_ARGS__);        \
        case 2: return FN<2, 1, 1, 0>(__VA_ARGS__);        \
        case 3: return FN<4, 1, 1, 0>(__VA_ARGS__);        \
        case 4: return FN<8, 1, 1, 0>(__VA_ARGS__);        \
        case 5: return FN<8, 1, 2, 0>(__VA_ARGS__);        \
        case 6: return FN<16, 1, 1, 0>(__VA_ARGS__);       \
        case 7: return FN<16, 1, 2, 0>(__VA_ARGS__);       \
        case 8: return FN<16, 1, 4, 0>(__VA_ARGS__);       \
        case 9: return FN<32, 1, 2, 0>(__VA_ARGS__);       \
        case 10: return FN<32, 1, 4, 0>(__VA_ARGS__);      \
        case 11: return FN<64, 1, 1, 0>(__VA_ARGS__);      \
        case 12: return FN<64, 1, 2, 0>(__VA_ARGS__);      \
        case 13: return FN<64, 1, 4, 0>(__VA_ARGS__);      \
        case 14: return FN<64, 1, 8, 0>(__VA_ARGS__);      \
        case 15: return FN<16, 4, 1, 0>(__VA_ARGS__);      \
        case 16: return FN<16, 4, 2, 0>(__VA_ARGS__);      \
        case 17: return FN<32, 2, 2, 0>(__VA_ARGS__);      \
        case 18: return FN<32, 2, 4, 0>(__VA_ARGS__);      \
        case 19: return FN<64, 2, 2, 0>(__VA_ARGS__);      \
        case 20: return FN<64, 2, 4, 0>(__VA_ARGS__);      \
        case 21: return FN<64, 4, 1, 0>(__VA_ARGS__);      \
        case 22: return FN<64, 4, 2, 0>(__VA_ARGS__);      \
        case 23: return FN<1, 1, 1, 1>(__VA_ARGS__);       \
        case 24: return FN<2, 1, 1, 1>(__VA_ARGS__);       \
        case 25: return FN<4, 1, 1, 1>(__VA_ARGS__);       \
        case 26: return FN<2, 4, 1, 0>(__VA_ARGS__);       \
        case 27: return FN<4, 2, 1, 0>(__VA_ARGS__);       \
        case 28: return FN<8, 1, 4, 0>(__VA_ARGS__);       \
        case 29: return FN<1, 2, 1, 1>(__VA_ARGS__);       \
        case 30: return FN<1, 4, 1, 1>(__VA_ARGS__);       \
        case 31: return FN<2, 4, 1, 1>(__VA_ARGS__);       \
        case 32: return FN<4, 2, 1, 1>(__VA_ARGS__);       \
        case 33: return FN<4, 4, 1, 0>(__VA_ARGS__);       \
        case 34: return FN<8, 4, 1, 0>(__VA_ARGS__);       \
        case 35: return FN<8, 2, 1, 0>(__VA_ARGS__);       \
        case 36: return FN##_nt<2, 0>(__VA_ARGS__);        \
        case 37: return FN##_nt<2, 1>(__VA_ARGS__);        \
        case 38: return FN<2, 1, 1, 0, 16>(__VA_ARGS__);   \
        case 39: return FN<4, 1, 1, 0, 16>(__VA_ARGS__);   \
        case 40: return FN##_nt<2, 0, 16>(__VA_ARGS__);    \
        case 41: return FN##_nt<2, 2, 16>(__VA_ARGS__);    \
        case 42: return FN##_nt<1, 2, 16>(__VA_ARGS__);    \
        default: return hipErrorInvalidValue;              \
    }

hipError_t launch_fwd(int sched, bool eval, const FwdArgs& A, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    HMS_SCHED_SWITCH(fwd_for, eval, A, blocks, s)
}

hipError_t launch_bwd(int sched, int opt, const BwdArgs& A, int blocks, hipStream_t s) {
    if (blocks <= 0) {
        // still advance the step counter
        if (opt != kGrad) {
            hipLaunchKernelGGL((k_bwd<1, 1, 1, kAdam, 0>), dim3(1), dim3(256), 0, s, A);
            return hipGetLastError();
        }
        return hipSuccess;
    }
    HMS_SCHED_SWITCH(bwd_for, opt, A, blocks, s)
}

hipError_t launch_combine(int opt, const BwdArgs& A, hipStream_t s) {
    const int64_t wide = (int64_t)A.n_heavy_wide * A.B.R;
    const int64_t narrow = (int64_t)(A.n_heavy - A.n_heavy_wide) * A.B.R;
    const int64_t blocks = wide + (narrow + 15) / 16;
    if (blocks == 0) return hipSuccess;
    if (opt == kAdam)
        hipLaunchKernelGGL((k_combine<kAdam>), dim3((int)blocks), dim3(1024), 0, s, A);
    else if (opt == kSgd)
        hipLaunchKernelGGL((k_combine<kSgd>), dim3((int)blocks), dim3(1024), 0, s, A);
    else
        hipLaunchKernelGGL((k_combine<kGrad>), dim3((int)blocks), dim3(1024), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_fwd_multi(int sched, bool eval, const MultiLaunch& M, hipStream_t s) {
    if (M.blocks <= 0) return hipSuccess;
    HMS_SCHED_SWITCH(fwd_multi_for, eval, M, s)
}

hipError_t launch_bwd_multi(int sched, int opt, const MultiLaunch& M, hipStream_t s) {
    if (M.blocks <= 0) return hipSuccess;
    if (opt != kAdam && opt != kSgd) return hipErrorInvalidValue;
    HMS_SCHED_SWITCH(bwd_multi_for, opt, M, s)
}

hipError_t launch_combine_multi(int opt, const MultiLaunch& M, hipStream_t s) {
    if (M.blocks <= 0) return hipSuccess;
    const BwdArgs* a = static_cast<const BwdArgs*>(M.args);
    if (opt == kAdam)
        hipLaunchKernelGGL((k_combine_multi<kAdam>), dim3(M.blocks), dim3(1024), 0, s, a, M.b0, M.n);
    else if (opt == kSgd)
        hipLaunchKernelGGL((k_combine_multi<kSgd>), dim3(M.blocks), dim3(1024), 0, s, a, M.b0, M.n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_reduce_multi(const MultiLaunch& stage1, const MultiLaunch& stage2, hipStream_t s) {
    const ReduceArgs* a1 = static_cast<const ReduceArgs*>(stage1.args);
    const ReduceArgs* a2 = static_cast<const ReduceArgs*>(stage2.args);
    if (stage1.blocks > 0) {
        hipLaunchKernelGGL(k_reduce1_multi, dim3(stage1.blocks), dim3(256), 0, s, a1, stage1.b0, stage1.n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (stage2.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_multi, dim3(stage2.blocks), dim3(1024), 0, s, a2, stage2.b0, stage2.n);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& A, hipStream_t s) {
    if (A.n_chunks > 0) {
        hipLaunchKernelGGL(k_reduce1, dim3((A.R + 63) / 64, A.n_chunks), dim3(256), 0, s, A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce, dim3((A.R + 63) / 64), dim3(1024), 0, s, A);
    return hipGetLastError();
}


hipError_t launch_build_slots(const SlotArgs& A, hipStream_t s) {
    if (A.c_ent_n <= 0) return hipSuccess;
    const int64_t fb = std::min<int64_t>((A.c_ent_n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_slot_fill, dim3((int)fb), dim3(256), 0, s, A.c_slot, A.c_ent_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || A.v_tiles == 0) return e;
    const int64_t rows = (int64_t)A.v_tiles * kTile;
    hipLaunchKernelGGL(k_slots, dim3((int)((rows + 255) / 256)), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_init(const InitArgs& A, hipStream_t s) {
    int64_t total = (int64_t)A.n * A.B.R;
    if (total < A.B.R) total = A.B.R;
    if (total < A.umask_words) total = A.umask_words;
    if (A.contrib != nullptr && total < A.contrib_n) total = A.contrib_n;
    if (total < 1) total = 1;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_snapshot(int32_t n_act, const Blocking& B, const float* x, const int32_t* improved,
                           uint8_t* best_a, hipStream_t s) {
    const int64_t total = (int64_t)n_act * B.R;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_snapshot, dim3((int)((total + 255) / 256)), dim3(256), 0, s, n_act, B, x, improved,
                       best_a);
    return hipGetLastError();
}

hipError_t launch_extract(int32_t n, const Blocking& B, int32_t r, const int32_t* var_old, const uint8_t* best_a,
                          uint8_t* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3((n + 255) / 256), dim3(256), 0, s, n, B, r, var_old, best_a, out);
    return hipGetLastError();
}

hipError_t launch_scatter_bytes(int32_t n, const Blocking& B, const int32_t* var_old, const uint8_t* src,
                                uint8_t* dst, hipStream_t s) {
    const int64_t total = (int64_t)n * B.R;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_bytes, dim3((int)((total + 255) / 256)), dim3(256), 0, s, n, B, var_old, src, dst);
    return hipGetLastError();
}

hipError_t launch_scatter(int32_t n, int32_t n_act, const Blocking& B, const int32_t* var_old, const float* src,
                          float* dst, hipStream_t s, const float* scale) {
    const int64_t total = (int64_t)n * B.R;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3((int)((total + 255) / 256)), dim3(256), 0, s, n, n_act, B, var_old, src,
                       dst, scale);
    return hipGetLastError();
}

}  // namespace hms
