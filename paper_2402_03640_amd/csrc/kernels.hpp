// Device kernels of the solve loop (gfx950, wave64).
//
// Data layout in HBM (n' = n + 1 rows, the last one a dummy variable whose
// relaxed value is -0.0; restart index innermost):
//   x, m, v, t : [n'][R] FP32   relaxed values, Adam moments, signed tanh(x)
//   a          : [c_tiles * 64 + 1][R] FP32   adjoint of the scores, last row 0
//   seg_part   : [seg_rows][R] FP64   partial transposed sums of heavy rows
//   cnt_part, loss_part : [units][R]   per-unit count / loss partials
//   best_a     : [n][R] bytes   rounded iterate of each restart's best step
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

struct FwdArgs {
    const TileDesc* tiles;
    const uint32_t* ent;
    int32_t ntiles, chunks, U, RG, R, all_mode;
    const float* t;
    float* a;
    float two_over_m;
    int32_t* cnt_part;
    double* loss_part;
    StepState* st;       // block 0 publishes the step scalars for the next update
    double lr, b1, b2;
};

struct BwdArgs {
    const TileDesc* tiles;
    const uint32_t* ent;
    int32_t ntiles, seg_tiles, chunks, U, RG, R;
    int32_t n_heavy, n_act, eval;
    const float* a;
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
    const int32_t* seg_row;
};

struct ReduceArgs {
    const int32_t* cnt_part;
    const double* loss_part;
    int32_t n_units, R, track;
    int64_t n_empty;
    double inv_m;
    int64_t* cur_count;
    double* cur_loss;
    int64_t* best;
    int32_t* best_step;
    int32_t* improved;
    const StepState* st;
};

struct InitArgs {
    int32_t n, R, a_zero_row, m;
    const int32_t* var_old;
    const float* x0;          // caller order [n][R] or null
    const uint8_t* assign0;   // caller order [n] (evaluate) or null
    uint64_t seed;
    float* x;
    float* t;
    float* mm;
    float* vv;
    float* a;
    uint8_t* best_a;
    int64_t* best;
    int32_t* best_step;
    int32_t* improved;
    StepState* st;
};

// Kernel schedules: P lanes per restart group (64 / P rows side by side),
// V restarts per lane (vector width), UR rows per lane handled together.
// A work unit is U rows of one tile (U a multiple of (64 / P) * UR dividing 64).
struct Schedule {
    int P, V, UR;
};
constexpr int kNumSchedules = 22;
extern const Schedule kSchedules[kNumSchedules + 1];

int default_rows_per_unit(int sched);

hipError_t launch_fwd(int sched, bool eval, const FwdArgs& A, int blocks, hipStream_t s);
hipError_t launch_bwd(int sched, int opt, const BwdArgs& A, int blocks, hipStream_t s);
hipError_t launch_combine(int opt, const BwdArgs& A, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& A, hipStream_t s);
hipError_t launch_init(const InitArgs& A, hipStream_t s);
hipError_t launch_snapshot(int32_t n_act, int32_t R, const float* x, const int32_t* improved,
                           uint8_t* best_a, hipStream_t s);
hipError_t launch_extract(int32_t n, int32_t R, int32_t r, const int32_t* var_old, const uint8_t* best_a,
                          uint8_t* out, hipStream_t s);
hipError_t launch_scatter(int32_t n, int32_t n_act, int32_t R, const int32_t* var_old, const float* src,
                          float* dst, hipStream_t s);

}  // namespace hms
