// Resident solver (see small.hpp).  The arithmetic is the same as the tiled
// kernels', operation for operation: clause scores summed over the tile's
// entries in plan order (FP64 for rows longer than 16), transposed sums over
// the variable rows in plan order in FP64, heavy rows by segment with the
// 64-slot combine tree, the same gradient and optimizer expressions.  So a
// resident solve is bitwise equal to the tiled one.
#include "small.hpp"

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "kernels.hpp"

namespace hms {

namespace {

// Adam step scalars are computed kScal steps ahead (the same FP64 expression
// as the tiled path), so no step waits on a pow.
constexpr int kScal = 1024;

struct SmallLds {
    float* t;      // [n + 1]
    float* a;      // [c_tiles * 64 + 1]
    float* x;      // [n]
    float* m;      // [n]
    float* v;      // [n]
    double* seg;   // [seg_rows]
};

__host__ __device__ __forceinline__ size_t align8(size_t b) { return (b + 7) & ~size_t(7); }
__host__ __device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// Byte size of one staged plan side: tile descriptors, then entries.
__host__ __device__ __forceinline__ size_t side_bytes(int32_t tiles, int64_t ents) {
    return align16((size_t)tiles * sizeof(TileDesc)) + align16((size_t)ents * 4);
}

// Reads of one plan side, from LDS when it is staged (S) and from global
// memory otherwise.  The address space is explicit so that the loads are LDS
// or global loads, not flat loads (which wait on both counters).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool S>
struct Side {
    const TileDesc* tiles;
    const uint32_t* ent;
    __device__ __forceinline__ TileDesc tile(int i) const {
        u32x4 q;
        if constexpr (S) q = ((const __attribute__((address_space(3))) u32x4*)tiles)[i];
        else q = ((const __attribute__((address_space(1))) u32x4*)tiles)[i];
        return TileDesc{q.x, q.y, q.z, q.w};
    }
    __device__ __forceinline__ uint32_t entry(size_t i) const {
        if constexpr (S) return ((const __attribute__((address_space(3))) uint32_t*)ent)[i];
        else return ((const __attribute__((address_space(1))) uint32_t*)ent)[i];
    }
};

// Copy one plan side into LDS (all kThreads threads); returns the bytes used.
template <int kThreads>
__device__ size_t stage_side(unsigned char* dst, const TileDesc* tiles, int32_t ntiles, const uint32_t* ent,
                             int64_t nent, const TileDesc*& tl, const uint32_t*& el) {
    TileDesc* t = reinterpret_cast<TileDesc*>(dst);
    for (int i = threadIdx.x; i < ntiles; i += kThreads) t[i] = tiles[i];
    uint32_t* e = reinterpret_cast<uint32_t*>(dst + align16((size_t)ntiles * sizeof(TileDesc)));
    for (int64_t i = threadIdx.x; i < nent; i += kThreads) e[i] = ent[i];
    tl = t;
    el = e;
    return side_bytes(ntiles, nent);
}

// Register-cached plan: a thread keeps the entries of its RF clause rows (up
// to FE entries each) and of its one variable row (up to kRegB) in registers
// for the whole solve.
constexpr int kRegB = 32;

// SC / SV: the clause / variable side is staged in LDS (for every instance of
// the launch).  NW wavefronts per workgroup: four when one pass of them covers
// every row (the barriers and the count reduction then cost less), else 16.
// RF > 0: the thread's rows' entries are kept in registers (RF clause rows of
// up to FE entries, one variable row), so a step reads only the relaxed values
// and adjoints from LDS.
template <bool SC, bool SV, int NW, int RF, int FE>
__global__ __launch_bounds__(NW * 64) void k_small(const SmallDesc* __restrict__ descs, int32_t n_desc) {
    constexpr int kThreads = NW * 64;
    constexpr int kWaves = NW;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t red_c[kWaves];
    __shared__ double red_l[kWaves];
    __shared__ float2 s_sc[kScal];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    // instance of this workgroup: the last descriptor with block0 <= blockIdx.x
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].block0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const SmallDesc& D = descs[lo];
    const int r = blockIdx.x - D.block0;
    const int n = D.n;
    const int crows = D.c_tiles * kTile;
    const int vrows = D.v_tiles * kTile;

    SmallLds L;
    size_t off = 0;
    L.t = reinterpret_cast<float*>(smem + off);
    off += (size_t)(n + 1) * 4;
    L.a = reinterpret_cast<float*>(smem + off);
    off += (size_t)(crows + 1) * 4;
    L.x = reinterpret_cast<float*>(smem + off);
    off += (size_t)n * 4;
    L.m = reinterpret_cast<float*>(smem + off);
    off += (size_t)n * 4;
    L.v = reinterpret_cast<float*>(smem + off);
    off += (size_t)n * 4;
    L.seg = reinterpret_cast<double*>(smem + align8(off));
    off = align16(align8(off) + (size_t)D.seg_rows * 8);
    // plan sides read every step: from LDS when staged, else global memory
    Side<SC> cs{D.c_tile, D.c_ent};
    Side<SV> vs{D.v_tile, D.v_ent};
    if constexpr (SC)
        off += stage_side<kThreads>(smem + off, D.c_tile, D.c_tiles, D.c_ent, D.c_ent_len, cs.tiles, cs.ent);
    if constexpr (SV)
        off += stage_side<kThreads>(smem + off, D.v_tile, D.v_tiles, D.v_ent, D.v_ent_len, vs.tiles, vs.ent);
    // every thread staged a strided share of the sides; the register cache
    // below reads other threads' shares
    if constexpr (SC || SV) __syncthreads();

    const AdamCoef co{D.b1, D.b2, D.eps, D.omb1, D.omb2};
    uint8_t* best_a = D.best_a + (size_t)r * n;

    // ---- initial point -------------------------------------------------------
    for (int i = tid; i < n; i += kThreads) {
        const int o = D.var_old[i];
        float x;
        if (D.x0 != nullptr) {
            x = D.x0[(size_t)o * D.R + r];
        } else {
            const uint64_t z = splitmix64(D.seed + (uint64_t)r, (uint64_t)o + 1);
            x = 2.0f * ((float)(z >> 40) * (1.0f / 16777216.0f)) - 1.0f;
        }
        L.x[i] = x;
        L.t[i] = signed_tanh(x);
        L.m[i] = D.m0 != nullptr ? D.m0[(size_t)o * D.R + r] : 0.0f;
        L.v[i] = D.v0 != nullptr ? D.v0[(size_t)o * D.R + r] : 0.0f;
        if (!D.resume) best_a[o] = x > 0.0f ? 1 : 0;
    }
    if (tid == 0) {
        L.t[n] = -0.0f;
        L.a[crows] = 0.0f;
    }
    // every thread tracks the best; thread 0's copy is stored at the end (a
    // resumed solve reads its entry values here, before the barriers below)
    int64_t best = D.resume ? D.best[r] : D.best0;
    int best_step = D.resume ? D.best_step[r] : -1;
    // with no split rows and at most one variable per thread, thread i owns
    // variable i (row i of the variable side): it keeps that variable's best
    // bit in a register and stores it once at the end
    const bool own = D.n_heavy == 0 && n <= kThreads;
    const int own_o = (own && tid < n) ? D.var_old[tid] : 0;
    bool own_bit = own && tid < n && (D.resume ? best_a[own_o] != 0 : L.x[tid] > 0.0f);

    // this thread's clause rows and variable row, entries in registers (RF >
    // 0); entries past a row's end are the padding entries, which add nothing.
    // A clause row's length, real and tautology flags are packed in fmeta;
    // the several-row caches serve unweighted instances only (weight 1).
    constexpr int kRF = RF > 0 ? RF : 1;
    constexpr int kFE = FE > 0 ? FE : 1;
    constexpr int kRW = RF == 1 ? 1 : 0;  // the one-row cache keeps the weight
    // the variable row is cached only beside a one-row clause cache (sixteen
    // wavefronts would run out of registers)
    constexpr int kRB = RF == 1 ? kRegB : 0;
    uint32_t fen[kRF][kFE], ben[kRB > 0 ? kRB : 1], fmeta[kRF];
    int64_t fw[kRW > 0 ? kRF : 1];
    uint32_t b_len = 0;
    bool b_real = false;
    if constexpr (RF > 0) {
#pragma unroll
        for (int q = 0; q < RF; ++q) {
            const int row = tid + q * kThreads;
            fmeta[q] = 0;
            if constexpr (kRW > 0) fw[q] = 1;
#pragma unroll
            for (int c = 0; c < FE; ++c) fen[q][c] = (uint32_t)n;
            if (row < crows) {
                const TileDesc d = cs.tile(row >> 6);
                const int rowin = row & 63;
                const bool real = rowin < (int)d.nreal;
                fmeta[q] = d.len | (real ? 1u << 8 : 0u) | ((d.flags & 1u) ? 1u << 9 : 0u);
                if constexpr (kRW > 0) fw[q] = (D.c_w != nullptr && real) ? D.c_w[row] : 1;
#pragma unroll
                for (int c = 0; c < FE; ++c)
                    if (c < (int)d.len) fen[q][c] = cs.entry((size_t)d.base + rowin + (size_t)c * kTile);
            }
        }
        if (kRB > 0 && tid < vrows) {
            const TileDesc d = vs.tile(tid >> 6);
            const int rowin = tid & 63;
            b_len = d.len;
            b_real = rowin < (int)d.nreal;
#pragma unroll
            for (int c = 0; c < kRB; ++c)
                ben[c] = c < (int)d.len ? vs.entry((size_t)d.base + rowin + (size_t)c * kTile) : (uint32_t)crows;
        }
    }
    __syncthreads();

    // parameters read every step, pinned in registers by an empty asm: left
    // as descriptor reads, the compiler re-issues the scalar loads inside the
    // loop, and each one's wait also waits for the LDS accesses in flight
    // (the values are uniform: readfirstlane moves them to scalar registers)
    int p_all = __builtin_amdgcn_readfirstlane(D.all_mode), p_opt = __builtin_amdgcn_readfirstlane(D.opt);
    int p_segt = __builtin_amdgcn_readfirstlane(D.seg_tiles), p_nh = __builtin_amdgcn_readfirstlane(D.n_heavy);
    int p_nact = __builtin_amdgcn_readfirstlane(D.n_act);
    int p_unw = __builtin_amdgcn_readfirstlane(D.c_w == nullptr ? 1 : 0);
    int p_tomb = __builtin_amdgcn_readfirstlane(__float_as_int(D.two_over_m));
    int p_lrb = __builtin_amdgcn_readfirstlane(__float_as_int(D.lr));
    int p_we0 = __builtin_amdgcn_readfirstlane((int)(uint32_t)D.w_empty);
    int p_we1 = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)D.w_empty >> 32));
    asm volatile("" : "+s"(p_all), "+s"(p_opt), "+s"(p_segt), "+s"(p_nh), "+s"(p_nact), "+s"(p_unw), "+s"(p_tomb),
                 "+s"(p_lrb), "+s"(p_we0), "+s"(p_we1));
    const float p_tom = __int_as_float(p_tomb), p_lr = __int_as_float(p_lrb);
    const int64_t p_wempty = (int64_t)(((uint64_t)(uint32_t)p_we1 << 32) | (uint32_t)p_we0);
    const int step0 = D.step0;  // iterations are numbered from here
    int kc = step0 % D.K;       // iteration number modulo K, kept by counting
    for (int step = 0; step <= D.T; ++step) {
        const bool eval = kc == 0 || step == D.T;
        if (++kc == D.K) kc = 0;
        // the loss is reported at x_T, and at every count when the trajectory is recorded
        const bool want_loss = step == D.T || (eval && D.trace != nullptr);
        if (p_opt != kSgd && step % kScal == 0 && step < D.T) {
            // the previous block of scalars is no longer read: the last step
            // ended with a barrier
            for (int k = tid; k < kScal && step + k < D.T; k += kThreads) {
                float ss, ib2;
                adam_scalars((double)(step0 + step + k) + 1.0, D.lr_d, D.b1_d, D.b2_d, ss, ib2);
                s_sc[k] = make_float2(ss, ib2);
            }
            __syncthreads();
        }
        // ---- clause scores, mask, adjoint ------------------------------------
        int64_t cnt = 0;
        double los = 0.0;
        // a clause row's outputs: adjoint, count and loss partials
        auto clause_out = [&](int row, float f, uint32_t allf, bool real, bool taut, int64_t wj) {
            const bool unsat = real && !taut && (allf >> 31) != 0;
            const bool mu = real && (p_all ? true : unsat);
            L.a[row] = mu ? (f * (float)wj) * p_tom : 0.0f;
            if (eval) {
                cnt += unsat ? wj : 0;
                if (want_loss) los += mu ? ((double)f * (double)f) * (double)wj : 0.0;
            }
        };
        if constexpr (RF > 0) {
#pragma unroll
            for (int q = 0; q < RF; ++q) {
                const int row = tid + q * kThreads;
                if (row < crows) {
                    const uint32_t len = fmeta[q] & 0xffu;
                    float f = 0.0f;
                    uint32_t allf = ~0u;
#pragma unroll
                    for (int c0 = 0; c0 < FE; c0 += 4)
                        if (c0 < (int)len) {
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const uint32_t en = fen[q][c0 + k];
                                const uint32_t b = __float_as_uint(L.t[en & kIdx]) ^ (en & kSign);
                                f = f + __uint_as_float(b);
                                allf &= b;
                            }
                        }
                    int64_t wj = 1;
                    if constexpr (kRW > 0) wj = fw[q];
                    clause_out(row, f, allf, (fmeta[q] >> 8) & 1u, (fmeta[q] >> 9) & 1u, wj);
                }
            }
        } else
        for (int row = tid; row < crows; row += kThreads) {
            const int tile = row >> 6;
            const int rowin = row & 63;
            const TileDesc d = cs.tile(tile);
            const size_t e = (size_t)d.base + rowin;
            float f = 0.0f;
            uint32_t allf = ~0u;
            if (d.len <= 16) {
#pragma unroll 4
                for (uint32_t c = 0; c < d.len; ++c) {
                    const uint32_t en = cs.entry(e + (size_t)c * kTile);
                    const uint32_t b = __float_as_uint(L.t[en & kIdx]) ^ (en & kSign);
                    f = f + __uint_as_float(b);
                    allf &= b;
                }
            } else {
                double fd = 0.0;
#pragma unroll 4
                for (uint32_t c = 0; c < d.len; ++c) {
                    const uint32_t en = cs.entry(e + (size_t)c * kTile);
                    const uint32_t b = __float_as_uint(L.t[en & kIdx]) ^ (en & kSign);
                    fd = fd + (double)__uint_as_float(b);
                    allf &= b;
                }
                f = (float)fd;
            }
            const bool real = rowin < (int)d.nreal;
            // clause weight (1 without weights), as in the tiled forward pass
            const int64_t wj = (!p_unw && real) ? D.c_w[row] : 1;
            clause_out(row, f, allf, real, (d.flags & 1u) != 0, wj);
        }
        if (eval) {
            if (p_unw) {
                // unweighted: each lane counts a few rows; the wavefront sum
                // is taken bit by bit with ballots, shorter than a shuffle tree
                uint32_t c32 = (uint32_t)cnt;
                int64_t tot = 0;
                for (int b = 0; __ballot(c32 != 0u) != 0ull; ++b) {
                    tot += (int64_t)__popcll(__ballot((c32 & 1u) != 0u)) << b;
                    c32 >>= 1;
                }
                cnt = tot;
            } else {
                for (int o2 = 32; o2 >= 1; o2 >>= 1) cnt += __shfl_xor(cnt, o2);
            }
            if (want_loss)
                for (int o2 = 32; o2 >= 1; o2 >>= 1) los += __shfl_xor(los, o2);
            if (lane == 0) {
                red_c[wave] = cnt;
                red_l[wave] = los;
            }
        }
        __syncthreads();
        if (eval) {
            // every thread sums the wavefront partials itself (the same exact
            // total everywhere) and keeps its own copy of the best, so no
            // second barrier has to broadcast the outcome; the partials are
            // rewritten only after the barrier that ends this step
            int64_t c = p_wempty;
            for (int w = 0; w < kWaves; ++w) c += red_c[w];
            const bool improved = c < best;
            if (improved) best = c;
            if (want_loss && tid == 0) {
                double l = 0.0;
                for (int w = 0; w < kWaves; ++w) l = l + red_l[w];
                if (step == D.T) D.final_loss[r] = l * D.inv_m;
                if (D.trace != nullptr) {
                    const int64_t gs = (int64_t)step0 + step;
                    const int64_t row = ((gs + D.K - 1) / D.K - ((int64_t)step0 + D.K - 1) / D.K) % D.trace_cap;
                    D.trace[(size_t)row * D.R + r] = TracePoint{(int32_t)gs, 0, c, l * D.inv_m};
                }
            }
            if (improved) {
                best_step = step0 + step;
                if (own) {
                    // only this thread writes x[tid] (in the transposed pass)
                    if (tid < n) own_bit = L.x[tid] > 0.0f;
                } else {
                    for (int i = tid; i < p_nact; i += kThreads) best_a[D.var_old[i]] = L.x[i] > 0.0f ? 1 : 0;
                    __syncthreads();
                }
            }
        }
        if (step == D.T) break;
        // ---- transposed sums, fused optimizer step ---------------------------
        const float2 sc = p_opt != kSgd ? s_sc[step % kScal] : make_float2(0.0f, 1.0f);
        const float ss = sc.x, ib2 = sc.y;
        // a variable row's outputs: a segment partial, or the gradient and the
        // optimizer step
        auto var_out = [&](int row, double G) {
            const int tile = row >> 6;
            if (tile < p_segt) {
                L.seg[row] = G;
            } else {
                const int var = p_nh + (row - p_segt * kTile);
                float x = L.x[var];
                const float g = grad_of(x, G);
                if (p_opt == kSgd) {
                    x = x - p_lr * g;
                } else {
                    float mm = L.m[var], vv = L.v[var];
                    adam_update(x, mm, vv, g, ss, ib2, co);
                    L.m[var] = mm;
                    L.v[var] = vv;
                }
                L.x[var] = x;
                L.t[var] = signed_tanh(x);
            }
        };
        if constexpr (kRB > 0) {
            if (tid < vrows && b_real) {
                double G = 0.0;
#pragma unroll
                for (int c0 = 0; c0 < kRB; c0 += 8)
                    if (c0 < (int)b_len) {
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const uint32_t en = ben[c0 + k];
                            G = G + (double)__uint_as_float(__float_as_uint(L.a[en & kIdx]) ^ (en & kSign));
                        }
                    }
                var_out(tid, G);
            }
        } else
        for (int row = tid; row < vrows; row += kThreads) {
            const int tile = row >> 6;
            const int rowin = row & 63;
            const TileDesc d = vs.tile(tile);
            if (rowin >= (int)d.nreal) continue;
            const size_t e = (size_t)d.base + rowin;
            double G = 0.0;
#pragma unroll 4
            for (uint32_t c = 0; c < d.len; ++c) {
                const uint32_t en = vs.entry(e + (size_t)c * kTile);
                G = G + (double)__uint_as_float(__float_as_uint(L.a[en & kIdx]) ^ (en & kSign));
            }
            var_out(row, G);
        }
        if (p_nh > 0) {
            __syncthreads();
            for (int h = wave; h < p_nh; h += kWaves) {
                double u = 0.0;
                const int p1 = D.seg_first[h + 1];
                for (int p = D.seg_first[h] + lane; p < p1; p += 64) u = u + L.seg[p];
#pragma unroll
                for (int o2 = 32; o2 >= 1; o2 >>= 1) u = u + __shfl_down(u, o2);
                if (lane == 0) {
                    float x = L.x[h];
                    const float g = grad_of(x, u);
                    if (p_opt == kSgd) {
                        x = x - p_lr * g;
                    } else {
                        float mm = L.m[h], vv = L.v[h];
                        adam_update(x, mm, vv, g, ss, ib2, co);
                        L.m[h] = mm;
                        L.v[h] = vv;
                    }
                    L.x[h] = x;
                    L.t[h] = signed_tanh(x);
                }
            }
        }
        __syncthreads();
    }
    if (own && tid < n) best_a[own_o] = own_bit ? 1 : 0;
    if (tid == 0) {
        D.best[r] = best;
        D.best_step[r] = best_step;
    }
    if (D.x_final != nullptr)
        for (int i = tid; i < n; i += kThreads) D.x_final[(size_t)D.var_old[i] * D.R + r] = L.x[i];
    if (D.m_final != nullptr)
        for (int i = tid; i < n; i += kThreads) {
            D.m_final[(size_t)D.var_old[i] * D.R + r] = L.m[i];
            D.v_final[(size_t)D.var_old[i] * D.R + r] = L.v[i];
        }
}

}  // namespace

size_t small_lds_bytes(const HostPlan& P) {
    size_t b = (size_t)(P.n + 1) * 4 + (size_t)(P.c_tiles * kTile + 1) * 4 + (size_t)P.n * 12;
    b = (b + 7) & ~size_t(7);
    b += (size_t)P.seg_rows * 8;
    return b;
}

size_t small_lds_total(const HostPlan& P, size_t limit, int32_t* stage) {
    size_t total = align16(small_lds_bytes(P));
    int32_t st = 0;
    const size_t cb = side_bytes(P.c_tiles, (int64_t)P.c_ent.size());
    const size_t vb = side_bytes(P.v_tiles, (int64_t)P.v_ent.size());
    if (total + cb <= limit) {
        st |= 1;
        total += cb;
    }
    if (total + vb <= limit) {
        st |= 2;
        total += vb;
    }
    if (stage) *stage = st;
    return total;
}

size_t small_static_lds() {
    hipFuncAttributes attr{};
    // the widest workgroup has the most static LDS (the per-wavefront partials)
    if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_small<true, true, 16, 0, 0>)) != hipSuccess) return 16384;
    return attr.sharedSizeBytes;
}

std::mutex g_attr_mu;  // serialises the one-time attribute settings below

// The dynamic-LDS attribute belongs to the kernel, not to the launch: it is
// set to the device's cap once per kernel and device, under a lock, before
// that kernel's first launch there, so no solve on another thread changes it
// while a launch of the kernel is being prepared.
template <bool SC, bool SV, int NW, int RF, int FE>
hipError_t launch_small_as(const SmallDesc* d_descs, int32_t n_desc, int32_t blocks, size_t lds_bytes, size_t lds_cap,
                           hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (lds_bytes > lds_cap) return hipErrorInvalidValue;
    static std::atomic<uint64_t> set_on{0};  // bit d: done on device d (< 64)
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev >= 0 && dev < 64 ? uint64_t(1) << dev : 0;
    if (!bit || !(set_on.load(std::memory_order_acquire) & bit)) {
        std::lock_guard<std::mutex> lk(g_attr_mu);
        if (!bit || !(set_on.load(std::memory_order_relaxed) & bit)) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small<SC, SV, NW, RF, FE>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cap);
            if (e != hipSuccess) return e;
            set_on.fetch_or(bit, std::memory_order_release);
        }
    }
    hipLaunchKernelGGL((k_small<SC, SV, NW, RF, FE>), dim3(blocks), dim3(NW * 64), lds_bytes, s, d_descs, n_desc);
    return hipGetLastError();
}

template <int NW, int RF, int FE>
hipError_t launch_small_nw(const SmallDesc* d_descs, int32_t n_desc, int32_t blocks, size_t lds_bytes, size_t lds_cap,
                           int32_t stage, hipStream_t s) {
    switch (stage & 3) {
        case 0: return launch_small_as<false, false, NW, RF, FE>(d_descs, n_desc, blocks, lds_bytes, lds_cap, s);
        case 1: return launch_small_as<true, false, NW, RF, FE>(d_descs, n_desc, blocks, lds_bytes, lds_cap, s);
        case 2: return launch_small_as<false, true, NW, RF, FE>(d_descs, n_desc, blocks, lds_bytes, lds_cap, s);
        default: return launch_small_as<true, true, NW, RF, FE>(d_descs, n_desc, blocks, lds_bytes, lds_cap, s);
    }
}

// Register-cache shapes: four wavefronts with one clause row of up to 16
// entries per thread, sixteen with up to kRF16 clause rows of up to 4.
constexpr int kRF4 = 1, kFE4 = 16;
constexpr int kRF16 = 5, kFE16 = 4;

int small_waves(int32_t rows) { return rows <= kSmallRows4 ? 4 : 16; }

bool small_reg_ok(const HostPlan& P, int32_t launch_rows) {
    const int32_t crows = P.c_tiles * kTile, vrows = P.v_tiles * kTile;
    const int nw = small_waves(launch_rows);
    const int rf = nw == 4 ? kRF4 : kRF16, fe = nw == 4 ? kFE4 : kFE16;
    if (crows > rf * nw * 64) return false;
    if (rf > 1 && P.weighted) return false;  // the several-row caches keep no weights
    for (const TileDesc& d : P.c_tile)
        if (d.len > (uint32_t)fe) return false;
    if (rf == 1) {  // the variable row is cached too
        if (vrows > nw * 64) return false;
        for (const TileDesc& d : P.v_tile)
            if (d.len > (uint32_t)kRegB) return false;
    }
    return true;
}

hipError_t launch_small(const SmallDesc* d_descs, int32_t n_desc, int32_t blocks, size_t lds_bytes, size_t lds_cap,
                        int32_t stage, int32_t rows, bool reg, hipStream_t s) {
    if (small_waves(rows) == 4) {
        if (reg) return launch_small_nw<4, kRF4, kFE4>(d_descs, n_desc, blocks, lds_bytes, lds_cap, stage, s);
        return launch_small_nw<4, 0, 0>(d_descs, n_desc, blocks, lds_bytes, lds_cap, stage, s);
    }
    if (reg) return launch_small_nw<16, kRF16, kFE16>(d_descs, n_desc, blocks, lds_bytes, lds_cap, stage, s);
    return launch_small_nw<16, 0, 0>(d_descs, n_desc, blocks, lds_bytes, lds_cap, stage, s);
}

}  // namespace hms
