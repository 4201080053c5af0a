// Resident solver: one workgroup runs the whole Algorithm 1 loop for one
// (instance, restart) with the relaxed state in LDS.  Used for instances whose
// state fits in LDS, where the tiled kernels would be bound by launch latency,
// and for batches of many such instances in one launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "plan.hpp"

namespace hms {

// One instance of a resident launch (device-visible, 256-byte aligned array).
struct SmallDesc {
    // plan (device)
    const TileDesc* c_tile;
    const uint32_t* c_ent;
    const TileDesc* v_tile;
    const uint32_t* v_ent;
    const int32_t* seg_first;
    const int32_t* var_old;
    const int64_t* c_w;   // weight of each clause row, or null (weight 1)
    int32_t n, m, n_act, n_heavy, c_tiles, v_tiles, seg_tiles, seg_rows;
    int64_t w_empty;      // weight of the empty clauses
    int64_t best0;        // initial best: the total clause weight
    int32_t c_ent_len, v_ent_len;
    int32_t stage;        // bit 0: clause tiles and entries fit in LDS beside the state, bit 1: variable side
    // solve parameters
    int32_t R, T, K, opt, all_mode, block0;
    float two_over_m;
    float lr, b1, b2, eps, omb1, omb2;
    double inv_m, lr_d, b1_d, b2_d;
    uint64_t seed;
    const float* x0;      // caller order [n][R] or null
    // resuming a solve (resume = 1): moments in caller order [n][R] (null:
    // zero); best_a, best and best_step below hold the resumed best on entry;
    // iterations are numbered from step0
    const float* m0;
    const float* v0;
    int32_t step0, resume;
    // outputs (device)
    uint8_t* best_a;      // [R][n] caller order: rounded iterate at each restart's best step
    int64_t* best;        // [R]
    int32_t* best_step;   // [R]
    double* final_loss;   // [R] loss at x_T
    float* x_final;       // caller order [n][R] or null
    float* m_final;       // caller order [n][R] or null: Adam moments after the last step
    float* v_final;
    TracePoint* trace;    // trajectory ring [trace_cap][R] or null (rows as in ReduceArgs)
    int32_t trace_cap;
};

// LDS bytes the resident solver needs for an instance's state (per workgroup).
size_t small_lds_bytes(const HostPlan& P);
// State plus the plan sides that also fit within `limit` bytes (clause side
// first), staged in LDS so the loop reads no plan data from global memory;
// *stage receives the SmallDesc::stage bits.
size_t small_lds_total(const HostPlan& P, size_t limit, int32_t* stage);
// LDS the resident kernel declares statically (on top of small_lds_bytes).
size_t small_static_lds();

// Launch one workgroup per (instance, restart): descs[i].block0 must be the
// running sum of the restart counts, `blocks` the total.  `stage` (SmallDesc
// bits) names the plan sides staged in LDS; every instance of the launch must
// have them (its stage bits include these).
// `rows` is the largest clause-side or variable-side row count (tiles * 64)
// among the launch's instances; it picks the wavefronts per workgroup: four
// when one pass of them covers every row (up to kSmallRows4), else sixteen.
constexpr int32_t kSmallRows4 = 256;
int small_waves(int32_t rows);
// True when the instance's rows fit the register cache of a launch whose
// largest instance has `launch_rows` rows (which fixes the wavefront count):
// with four wavefronts one clause row of up to 16 entries and one variable row
// of up to 32 per thread; with sixteen, unweighted, up to five clause rows of
// up to 4 entries per thread (the variable side stays in LDS).
// `reg` of a launch must hold for every instance in it.
bool small_reg_ok(const HostPlan& P, int32_t launch_rows);
// `lds_cap` is the device's dynamic-LDS cap (the same on every call for one
// device); lds_bytes above it is an invalid value.
hipError_t launch_small(const SmallDesc* d_descs, int32_t n_desc, int32_t blocks, size_t lds_bytes, size_t lds_cap,
                        int32_t stage, int32_t rows, bool reg, hipStream_t s);

}  // namespace hms
