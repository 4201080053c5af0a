// Device kernels of the solve loop (gfx950, wave64).
//
// Data layout in HBM.  Restarts are stored in groups of G (blocked layout):
// element (row, r) of an array with `rows` rows sits at
//     ((r / G) * rows + row) * G + (r % G).
// G is the number of restarts one wavefront group covers (P lanes x V), so a
// gather of one row for one group is one contiguous run of G floats, and a
// workgroup works on a single restart group chosen as blockIdx % RG.  Since
// workgroups are dispatched round-robin over the 8 XCDs, with RG = 8 each XCD
// only touches its own restart slice, which stays in that XCD's L2.
//   x, m, v, t : [RG][n + 1][G] FP32   relaxed values, Adam moments, signed tanh(x)
//                (row n is a dummy variable whose t is -0.0: the padding literal)
//   a          : [RG][c_tiles * 64 + 1][G] FP32   adjoint of the scores (last row 0)
//   seg_part   : [RG][seg_rows][G] FP64   partial transposed sums of heavy rows
//   best_a     : [RG][n + 1][G] bytes     rounded iterate at each restart's best step
//   cnt_part, loss_part : [units][R]     per-unit unsatisfied weight (int64) / loss partials
//   umask      : [RG][c_tiles * 2 + 1] bitset words over clause rows: bit j of group g =
//                clause j unsatisfied for some restart of group g (unsat-masked loss)
//   contrib    : [v_ent entries] FP32, slot schedules only (one restart, unsat-masked
//                loss): the signed adjoint of each occurrence, at the index of its
//                variable-side entry, 0 for clauses outside the loss
//
// t stores tanh(x) with its sign bit forced to "x does not round to true":
// sign(t) = 1 iff !(x > 0).  A literal entry holds the variable index and the
// literal's sign in bit 31; xor-ing that bit into t gives the signed term
// sigma * tanh(x) whose sign bit is set exactly when the literal is false.  A
// clause is unsatisfied iff all its terms have the sign bit set, and its score
// is the sum of the terms.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace hms {

enum OptKind : int32_t { kAdam = 0, kSgd = 1, kGrad = 2 };

struct StepState {
    int32_t t;           // index of the current iterate x_t
    int32_t pad;
    float step_size;     // lr / (1 - beta1^(t+1))
    float inv_sqrt_bc2;  // 1 / sqrt(1 - beta2^(t+1))
};

// Restart blocking shared by all kernels of one solve.
struct Blocking {
    int32_t R, G, RG;   // restarts, group width, groups
    int32_t rows_x;     // n + 1
    int32_t rows_a;     // c_tiles * 64 + 1
    int32_t rows_seg;   // max(seg_rows, 1)
};

struct FwdArgs {
    const TileDesc* tiles;
    const uint32_t* ent;
    uint32_t pad_entry;  // entry standing for "no literal" (the dummy variable)
    int32_t ntiles, chunks, U, all_mode;
    int32_t umask_words; // bitset words per restart group
    Blocking B;
    const float* t;
    float* a;
    uint32_t* umask;     // written when the schedule keeps the unsat bitset
    const int64_t* w;    // weight of each clause row (weighted MaxSAT), or null: weight 1
    const uint32_t* slot; // slot schedules: variable-side entry of each clause-side entry | sign
                          // (tile-major like the entries, but row by row within a tile)
    float* contrib;       // slot schedules: occurrence adjoints (written where they change)
    float two_over_m;
    int64_t* cnt_part;   // unsatisfied weight per unit
    double* loss_part;
    StepState* st;       // block 0 publishes the step scalars for the next update
    double lr, b1, b2;
};

struct BwdArgs {
    const TileDesc* tiles;
    const uint32_t* ent;
    uint32_t pad_entry;  // entry standing for "no occurrence" (the zero adjoint row)
    int32_t ntiles, seg_tiles, chunks, U;
    Blocking B;
    int32_t n_heavy, n_heavy_wide, n_act, eval;
    int32_t umask_words; // bitset words per restart group
    const float* a;
    const uint32_t* umask;
    const float* contrib; // slot schedules: occurrence adjoints, parallel to ent
    double* seg_part;
    float* x;
    float* m;
    float* v;
    float* t;
    float* g_out;
    uint8_t* best_a;
    const int32_t* improved;
    StepState* st;
    float lr, b1, b2, eps, omb1, omb2;
    const int32_t* seg_first;
};

// One counted iterate of one restart: the trajectory record of a solve.
struct TracePoint {
    int32_t step, pad;
    int64_t cost;
    double loss;
};

struct ReduceArgs {
    const int64_t* cnt_part;
    const double* loss_part;
    int64_t* cnt_mid;        // [n_chunks][R] stage-1 partials
    double* loss_mid;
    int32_t n_units, chunk, n_chunks, R, track;
    int64_t n_empty;         // weight of the empty clauses (always unsatisfied)
    double inv_m;
    int64_t* cur_count;
    double* cur_loss;
    int64_t* best;
    int32_t* best_step;
    int32_t* improved;
    const StepState* st;
    // trajectory ring (or null): the count at iteration t goes to row
    // (ceil(t / trace_k) - trace_base) % trace_cap of [trace_cap][R]
    TracePoint* trace;
    int32_t trace_cap, trace_k, trace_base;
};

struct InitArgs {
    int32_t n, m, a_zero_row, umask_words;
    int64_t best0;            // initial best: the total clause weight (m without weights)
    Blocking B;
    const int32_t* var_old;
    const float* x0;          // caller order [n][R] or null
    const uint8_t* assign0;   // caller order [n] (evaluate) or null
    // resuming a solve: moments in caller order [n][R] (null: zero), best
    // rounded iterates in caller order [R][n] (null: round(x0)), the step count
    // to continue from, and keep_best = 1 when best / best_step already hold
    // the resumed values (uploaded before this kernel)
    const float* m0;
    const float* v0;
    const uint8_t* best_a0;
    int32_t step0, keep_best;
    uint64_t seed;
    float* x;
    float* t;
    float* mm;
    float* vv;
    float* a;
    uint32_t* umask;
    float* contrib;           // slot schedules: zeroed (contrib_n floats), else null
    int64_t contrib_n;
    uint8_t* best_a;
    int64_t* best;
    int32_t* best_step;
    int32_t* improved;
    StepState* st;
};

// Kernel schedules: P lanes per restart group (64 / P rows side by side),
// V restarts per lane (vector width), UR rows per lane handled together.
// A work unit is U rows of one tile (U a multiple of (64 / P) * UR dividing 64).
// MASK schedules (unsat-masked loss only) keep the unsat bitset and skip the
// adjoint gathers of clauses satisfied in every restart of the group; they
// need U >= 32 and UR = 1.  `twin` is the schedule with the same arithmetic
// and no bitset that runs in their place when the loss is not masked.
// Slot schedules (one restart, unsat-masked loss) have the forward write each
// occurrence's signed adjoint into the slot parallel to its variable-side
// entry, for the clauses in the loss and those that just left it, so the
// backward reads its terms in entry order with no gather; they fall back to
// `twin` elsewhere.  The terms and their order are those of every schedule.
struct Schedule {
    int P, V, UR, mask, twin;
    int nt = 1;    // whole clause tiles per forward wavefront (more than 1 only with P = V = UR = 1;
                   // slot schedules always take whole tiles)
    int cb = 8;    // columns per backward load batch (16 only with V = UR = 1)
    int slot = 0;  // slot schedule
};
constexpr int kNumSchedules = 42;
extern const Schedule kSchedules[kNumSchedules + 1];

int default_rows_per_unit(int sched);

hipError_t launch_fwd(int sched, bool eval, const FwdArgs& A, int blocks, hipStream_t s);
hipError_t launch_bwd(int sched, int opt, const BwdArgs& A, int blocks, hipStream_t s);
hipError_t launch_combine(int opt, const BwdArgs& A, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& A, hipStream_t s);

// One launch over many instances: `args` is a device array of n argument
// structs (FwdArgs, BwdArgs or ReduceArgs), instance i owns workgroups
// [b0[i], b0[i+1]) of a `blocks`-workgroup grid (b0: device, n + 1 entries).
// Every instance runs exactly what its own launch would.
struct MultiLaunch {
    const void* args;
    const int32_t* b0;
    int32_t n, blocks;
};
hipError_t launch_fwd_multi(int sched, bool eval, const MultiLaunch& M, hipStream_t s);
hipError_t launch_bwd_multi(int sched, int opt, const MultiLaunch& M, hipStream_t s);
hipError_t launch_combine_multi(int opt, const MultiLaunch& M, hipStream_t s);
// Stage 1 (grids ceil(R/64) x n_chunks, flattened) then stage 2 (ceil(R/64)).
hipError_t launch_reduce_multi(const MultiLaunch& stage1, const MultiLaunch& stage2, hipStream_t s);
// The clause-side -> variable-side occurrence map of the slot schedules,
// built on the device at load: c_slot[clause-side entry] = variable-side
// entry of the same occurrence | its sign bit, kNoSlot for padding.
struct SlotArgs {
    const TileDesc* c_tile;
    const uint32_t* c_ent;
    const TileDesc* v_tile;
    const uint32_t* v_ent;
    const int32_t* seg_first;  // [n_heavy + 1] first segment row of each heavy variable
    int32_t n_heavy, seg_rows, seg_tiles, v_tiles;
    uint32_t vpad;             // variable-side padding entry
    uint32_t* c_slot;
    int64_t c_ent_n;
};
hipError_t launch_build_slots(const SlotArgs& A, hipStream_t s);

hipError_t launch_init(const InitArgs& A, hipStream_t s);
hipError_t launch_snapshot(int32_t n_act, const Blocking& B, const float* x, const int32_t* improved,
                           uint8_t* best_a, hipStream_t s);
hipError_t launch_extract(int32_t n, const Blocking& B, int32_t r, const int32_t* var_old, const uint8_t* best_a,
                          uint8_t* out, hipStream_t s);
// dst[r][var_old[i]] = src(i, r) for the blocked bytes src (a restart's
// best rounded iterate in caller order, one row per restart).
hipError_t launch_scatter_bytes(int32_t n, const Blocking& B, const int32_t* var_old, const uint8_t* src,
                                uint8_t* dst, hipStream_t s);
// dst[var_old[i]][r] = scale[r] * src(i, r) (scale may be null: 1), 0 for inactive variables.
hipError_t launch_scatter(int32_t n, int32_t n_act, const Blocking& B, const int32_t* var_old, const float* src,
                          float* dst, hipStream_t s, const float* scale = nullptr);

}  // namespace hms
