// C ABI of the solve loop: instance loading, Algorithm 1 driver, evaluation.
// Host code; the kernels are in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hipmsat.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "small.hpp"

struct hms_cnf {
    hms::HostPlan plan;
    int device = -1;
    void* arena = nullptr;
    hms::TileDesc* c_tile = nullptr;
    uint32_t* c_ent = nullptr;
    uint32_t* c_slot = nullptr;  // variable-side entry of each clause-side entry (slot schedules)
    hms::TileDesc* v_tile = nullptr;
    uint32_t* v_ent = nullptr;
    int32_t* seg_first = nullptr;
    int32_t* var_old = nullptr;
    int64_t* c_w = nullptr;  // clause-row weights (weighted instances only)
    int64_t struct_bytes = 0;
    // autotuned schedule per (restarts, optimizer, loss mode); results do not
    // depend on the schedule, only the speed does
    mutable std::mutex tune_mu;
    mutable std::map<uint64_t, int32_t> tuned;
};

namespace {

thread_local std::string g_err;

hms_status fail(hms_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPTRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? HMS_ERR_NOMEM : HMS_ERR_DEVICE,                \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

// Bump layout of one device allocation (256-byte aligned pieces).
struct Layout {
    size_t off = 0;
    size_t add(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

hms_status current_gfx950(int& dev) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("no HIP device available: ") + hipGetErrorString(e));
    if (count == 0) return fail(HMS_ERR_DEVICE, "no HIP device available");
    HIPTRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPTRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HMS_ERR_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library targets gfx950");
    return HMS_OK;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Stream-ordered scratch arena, released on scope exit (owns = false: a
// view of memory the arena does not own, never freed).
struct Arena {
    char* base = nullptr;
    hipStream_t s = nullptr;
    bool owns = true;
    ~Arena() {
        if (base && owns) (void)hipFreeAsync(base, s);
    }
    template <typename T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(base + off);
    }
};

// Waits for the stream when it goes out of scope: declared right after an
// asynchronous copy from a host buffer, it keeps an early error return from
// freeing that buffer while the copy may still read it.
struct SyncOnExit {
    hipStream_t s;
    bool on = true;  // false: nothing to wait for
    ~SyncOnExit() {
        if (on) (void)hipStreamSynchronize(s);
    }
};

// Default kernel schedule for R restarts (table index into hms::kSchedules).
// One restart: above 2^20 nonzeros (unsat-masked loss) one row per lane with
// the unsat bitset and two clause tiles per forward wavefront (entry 37);
// below, 16-column backward batches (half the round trips of a long row),
// with four lanes per row up to 2^14 active variables (entry 39: one of them
// works, so a wavefront takes 16 rows and a small instance's rows spread over
// four times the wavefronts), else two (entry 38).
int auto_schedule(int32_t R, int loss_mode, int64_t nnz = 0, int32_t n_act = 0) {
    if (R <= 1) {
        // the slot schedules from 2^17 nonzeros with the unsat-masked loss:
        // two clause tiles per forward wavefront past 2^22, one below
        if (loss_mode == HMS_LOSS_UNSAT && nnz > (1 << 22)) return 41;
        if (loss_mode == HMS_LOSS_UNSAT && nnz > (1 << 17)) return 42;
        if (loss_mode != HMS_LOSS_UNSAT && nnz > (1 << 20)) return 36;
        // long backward batches; four lanes per variable row (more wavefronts)
        // while the rows are few, two beyond
        return n_act <= (1 << 14) ? 39 : 38;
    }
    if (R <= 2) return 2;
    if (R <= 4) return 3;
    if (R <= 8) return 5;
    if (R <= 16) return 4;
    if (R <= 32) return 10;
    if (R % 4 == 0) return 15;
    return 14;
}

struct Shape {
    int sched, P, V, UR, U, chunks, mask, nt, slot;
    int Ub, chunks_b;  // rows per work unit and units per tile of the backward pass
    hms::Blocking B;
    int64_t n_tc, fwd_blocks64, bwd_blocks64;
    int fwd_blocks, bwd_blocks;
    int32_t code;  // schedule id as reported: table index | U << 8
};

// Schedule id: bits 0..7 = table index (0 = automatic), bits 8..15 = rows per
// work unit U (0 = the default for that entry), bits 16..23 = rows per work
// unit of the backward pass (0 = U).  The bitset variants apply to
// the unsat-masked loss; elsewhere they fall back to their unmasked twin (same
// arithmetic).
hms_status make_shape(const hms::HostPlan& P, int32_t R, int32_t req, int loss_mode, Shape& sh,
                      bool allow_mask = true, bool allow_slot = true) {
    const int idx = req & 0xff;
    int U = (req >> 8) & 0xff;
    int Ub = (req >> 16) & 0xff;
    if (req < 0 || (req >> 24) != 0 || idx > hms::kNumSchedules) return fail(HMS_ERR_ARG, "unknown schedule id");
    sh.sched = idx == 0 ? auto_schedule(R, loss_mode, P.nnz, P.n_act) : idx;
    if (hms::kSchedules[sh.sched].mask && (loss_mode != HMS_LOSS_UNSAT || !allow_mask))
        sh.sched = hms::kSchedules[sh.sched].twin;
    // slot schedules: one restart, the unsat-masked loss, and a plan with the
    // occurrence map; elsewhere their twin
    if (hms::kSchedules[sh.sched].slot &&
        (R != 1 || loss_mode != HMS_LOSS_UNSAT || !allow_mask || !allow_slot || !P.slot_ok))
        sh.sched = hms::kSchedules[sh.sched].twin;
    const hms::Schedule& c = hms::kSchedules[sh.sched];
    sh.P = c.P;
    sh.V = c.V;
    sh.UR = c.UR;
    sh.mask = c.mask;
    sh.slot = c.slot;
    if (R % sh.V != 0) return fail(HMS_ERR_ARG, "schedule vector width does not divide the restart count");
    if (U == 0) U = hms::default_rows_per_unit(sh.sched);
    if (Ub == 0) Ub = U;
    const int per_pass = (64 / sh.P) * sh.UR;
    if (U % per_pass != 0 || hms::kTile % U != 0 || (sh.mask && U < 32) || Ub % per_pass != 0 || hms::kTile % Ub != 0)
        return fail(HMS_ERR_ARG, "rows per unit must be a multiple of the rows per pass and divide 64");
    sh.nt = c.nt;  // whole clause tiles per forward work unit (rows per unit then stay 64)
    sh.U = U;
    sh.Ub = Ub;
    sh.code = sh.sched | (U << 8) | (Ub != U ? Ub << 16 : 0);
    sh.chunks = hms::kTile / sh.U;
    sh.chunks_b = hms::kTile / sh.Ub;
    int G = sh.P * sh.V;
    int Rp = 1;
    while (Rp < R && Rp < G) Rp <<= 1;
    G = std::min(G, Rp);
    sh.B.R = R;
    sh.B.G = G;
    sh.B.RG = (R + G - 1) / G;
    sh.B.rows_x = P.n + 1;
    sh.B.rows_a = P.a_rows();
    sh.B.rows_seg = std::max(P.seg_rows, 1);
    sh.n_tc = sh.nt > 1 ? ((int64_t)P.c_tiles + sh.nt - 1) / sh.nt : (int64_t)P.c_tiles * sh.chunks;
    const int64_t n_vu = (int64_t)P.v_tiles * sh.chunks_b;
    sh.fwd_blocks64 = (int64_t)sh.B.RG * ((sh.n_tc + 3) / 4);
    sh.bwd_blocks64 = (int64_t)sh.B.RG * ((n_vu + 3) / 4);
    if (sh.fwd_blocks64 >= INT32_MAX / 2 || sh.bwd_blocks64 >= INT32_MAX / 2)
        return fail(HMS_ERR_TOO_LARGE, "too many work units");
    sh.fwd_blocks = (int)sh.fwd_blocks64;
    sh.bwd_blocks = (int)sh.bwd_blocks64;
    return HMS_OK;
}

// Device buffers of one solve / evaluation.
struct State {
    float *x, *m, *v, *t, *a, *g;
    double* seg_part;
    int64_t* cnt_part;
    double* loss_part;
    uint8_t* best_a;
    uint32_t* umask;
    int64_t *best, *cur_count;
    int32_t *best_step, *improved;
    double* cur_loss;
    int64_t* cnt_mid;
    double* loss_mid;
    hms::StepState* st;
    uint8_t* out_assign;
    float* contrib;  // slot schedules
};

enum { kOffX, kOffM, kOffV, kOffT, kOffA, kOffG, kOffSeg, kOffCnt, kOffLoss, kOffBest, kOffMask, kOffBestC,
       kOffCurC, kOffBestS, kOffImp, kOffCurL, kOffCntMid, kOffLossMid, kOffSt, kOffContrib, kOffN };
constexpr size_t kNoOff = ~size_t(0);  // a piece the solve does not have

// Units per stage-1 reduce chunk: a fixed function of the unit count.
int32_t reduce_chunk(int64_t n_units) { return (int32_t)std::max<int64_t>(64, (n_units + 1023) / 1024); }
// Stage-1 chunks of the count/loss reduction; 0 when the final stage can sum
// the unit partials itself with at most 16 loads per thread (its 1024 threads
// hold `restart lanes` restarts side by side), which saves a launch.
int32_t reduce_chunks(int64_t n_units, int32_t R) {
    int64_t rp = 1;
    while (rp < 64 && rp < R) rp <<= 1;
    if (n_units * rp <= 16 * 1024) return 0;
    return (int32_t)((n_units + reduce_chunk(n_units) - 1) / reduce_chunk(n_units));
}

int32_t umask_words(const hms::HostPlan& P) { return P.c_tiles * 2 + 1; }

void layout_state(const hms::HostPlan& P, const Shape& sh, bool moments, bool grad, bool best, Layout& L,
                  size_t off[kOffN]) {
    const int32_t R = sh.B.R;
    const size_t Rp = (size_t)sh.B.RG * sh.B.G;  // padded restart count of the blocked layout
    const size_t nR = (size_t)sh.B.rows_x * Rp;
    off[kOffX] = L.add(nR * 4);
    off[kOffM] = moments ? L.add(nR * 4) : 0;
    off[kOffV] = moments ? L.add(nR * 4) : 0;
    off[kOffT] = L.add(nR * 4);
    off[kOffA] = L.add((size_t)sh.B.rows_a * Rp * 4);
    off[kOffG] = grad ? L.add(nR * 4) : 0;
    off[kOffSeg] = L.add((size_t)sh.B.rows_seg * Rp * 8);
    off[kOffCnt] = L.add((size_t)std::max<int64_t>(sh.n_tc, 1) * R * 8);
    off[kOffLoss] = L.add((size_t)std::max<int64_t>(sh.n_tc, 1) * R * 8);
    off[kOffBest] = best ? L.add(nR) : 0;
    off[kOffMask] = L.add((size_t)umask_words(P) * sh.B.RG * 4);
    off[kOffBestC] = L.add((size_t)R * 8);
    off[kOffCurC] = L.add((size_t)R * 8);
    off[kOffBestS] = L.add((size_t)R * 4);
    off[kOffImp] = L.add((size_t)R * 4);
    off[kOffCurL] = L.add((size_t)R * 8);
    off[kOffCntMid] = L.add((size_t)std::max(reduce_chunks(sh.n_tc, R), 1) * R * 8);
    off[kOffLossMid] = L.add((size_t)std::max(reduce_chunks(sh.n_tc, R), 1) * R * 8);
    off[kOffSt] = L.add(256 + (size_t)std::max(P.n, 1));  // step state, then out_assign at +256
    off[kOffContrib] = sh.slot ? L.add(P.v_ent.size() * 4) : kNoOff;
}

State bind_state(const Arena& A, const size_t off[kOffN], bool moments, bool grad, bool best) {
    State S{};
    S.x = A.at<float>(off[kOffX]);
    S.m = moments ? A.at<float>(off[kOffM]) : nullptr;
    S.v = moments ? A.at<float>(off[kOffV]) : nullptr;
    S.t = A.at<float>(off[kOffT]);
    S.a = A.at<float>(off[kOffA]);
    S.g = grad ? A.at<float>(off[kOffG]) : nullptr;
    S.seg_part = A.at<double>(off[kOffSeg]);
    S.cnt_part = A.at<int64_t>(off[kOffCnt]);
    S.loss_part = A.at<double>(off[kOffLoss]);
    S.best_a = best ? A.at<uint8_t>(off[kOffBest]) : nullptr;
    S.umask = A.at<uint32_t>(off[kOffMask]);
    S.best = A.at<int64_t>(off[kOffBestC]);
    S.cur_count = A.at<int64_t>(off[kOffCurC]);
    S.best_step = A.at<int32_t>(off[kOffBestS]);
    S.improved = A.at<int32_t>(off[kOffImp]);
    S.cur_loss = A.at<double>(off[kOffCurL]);
    S.cnt_mid = A.at<int64_t>(off[kOffCntMid]);
    S.loss_mid = A.at<double>(off[kOffLossMid]);
    S.st = A.at<hms::StepState>(off[kOffSt]);
    S.out_assign = A.at<uint8_t>(off[kOffSt] + 256);
    S.contrib = off[kOffContrib] != kNoOff ? A.at<float>(off[kOffContrib]) : nullptr;
    return S;
}

hms::InitArgs make_init(const hms_cnf* C, const Shape& sh, const State& S) {
    const hms::HostPlan& P = C->plan;
    hms::InitArgs ia{};
    ia.n = P.n;
    ia.m = P.m;
    ia.a_zero_row = P.a_zero_row();
    ia.umask_words = umask_words(P) * sh.B.RG;
    ia.best0 = P.w_total;
    ia.B = sh.B;
    ia.var_old = C->var_old;
    ia.x = S.x;
    ia.t = S.t;
    ia.mm = S.m;
    ia.vv = S.v;
    ia.a = S.a;
    ia.umask = S.umask;
    ia.contrib = S.contrib;
    ia.contrib_n = S.contrib ? (int64_t)P.v_ent.size() : 0;
    ia.best_a = S.best_a;
    ia.st = S.st;
    if (S.best_a) {
        ia.best = S.best;
        ia.best_step = S.best_step;
        ia.improved = S.improved;
    }
    return ia;
}

struct Launch {
    hms::FwdArgs fa;
    hms::BwdArgs ba;
    hms::ReduceArgs ra;
    Shape sh;
    int opt;
};

Launch make_launch(const hms_cnf* C, const Shape& sh, const State& S, int opt, int loss_mode, float lr, float b1,
                   float b2, float eps) {
    const hms::HostPlan& P = C->plan;
    Launch L{};
    L.sh = sh;
    L.opt = opt;
    hms::FwdArgs& f = L.fa;
    f.tiles = C->c_tile;
    f.ent = C->c_ent;
    f.pad_entry = (uint32_t)P.n;
    f.ntiles = P.c_tiles;
    f.chunks = sh.chunks;
    f.U = sh.U;
    f.all_mode = loss_mode == HMS_LOSS_ALL;
    f.B = sh.B;
    f.t = S.t;
    f.a = S.a;
    f.umask = S.umask;
    f.umask_words = umask_words(P);
    f.w = C->c_w;
    f.slot = C->c_slot;
    f.contrib = S.contrib;
    f.two_over_m = P.m > 0 ? (float)(2.0 / (double)P.m) : 0.0f;
    f.cnt_part = S.cnt_part;
    f.loss_part = S.loss_part;
    f.st = S.st;
    f.lr = lr;
    f.b1 = b1;
    f.b2 = b2;
    hms::BwdArgs& b = L.ba;
    b.tiles = C->v_tile;
    b.ent = C->v_ent;
    b.pad_entry = (uint32_t)P.a_zero_row();
    b.ntiles = P.v_tiles;
    b.seg_tiles = P.seg_tiles;
    b.chunks = sh.chunks_b;
    b.U = sh.Ub;
    b.B = sh.B;
    b.n_heavy = P.n_heavy;
    b.n_heavy_wide = P.n_heavy_wide;
    b.n_act = P.n_act;
    b.eval = 0;
    b.a = S.a;
    b.umask = S.umask;
    b.umask_words = umask_words(P);
    b.contrib = S.contrib;
    b.seg_part = S.seg_part;
    b.x = S.x;
    b.m = S.m;
    b.v = S.v;
    b.t = S.t;
    b.g_out = S.g;
    b.best_a = S.best_a;
    b.improved = S.improved;
    b.st = S.st;
    b.lr = lr;
    b.b1 = b1;
    b.b2 = b2;
    b.eps = eps;
    b.omb1 = 1.0f - b1;
    b.omb2 = 1.0f - b2;
    b.seg_first = C->seg_first;
    hms::ReduceArgs& r = L.ra;
    r.cnt_part = S.cnt_part;
    r.loss_part = S.loss_part;
    r.n_units = (int32_t)sh.n_tc;
    r.chunk = reduce_chunk(sh.n_tc);
    r.n_chunks = reduce_chunks(sh.n_tc, sh.B.R);
    r.cnt_mid = S.cnt_mid;
    r.loss_mid = S.loss_mid;
    r.R = sh.B.R;
    r.track = 1;
    r.n_empty = P.w_empty;
    r.inv_m = P.m > 0 ? 1.0 / (double)P.m : 0.0;
    r.cur_count = S.cur_count;
    r.cur_loss = S.cur_loss;
    r.best = S.best;
    r.best_step = S.best_step;
    r.improved = S.improved;
    r.st = S.st;
    return L;
}

// One step of Algorithm 1 on stream s.
hipError_t enqueue_step(const Launch& L, bool eval, hipStream_t s) {
    hipError_t e = hms::launch_fwd(L.sh.sched, eval, L.fa, L.sh.fwd_blocks, s);
    if (e != hipSuccess) return e;
    if (eval) {
        e = hms::launch_reduce(L.ra, s);
        if (e != hipSuccess) return e;
    }
    hms::BwdArgs b = L.ba;
    b.eval = eval ? 1 : 0;
    e = hms::launch_bwd(L.sh.sched, L.opt, b, L.sh.bwd_blocks, s);
    if (e != hipSuccess) return e;
    return hms::launch_combine(L.opt, b, s);
}

hms_status check_cnf(const hms_cnf* C) {
    if (!C) return fail(HMS_ERR_ARG, "null instance handle");
    return HMS_OK;
}

template <typename T>
hms_status upload(const hms::PVec<T>& h, T* d, hipStream_t s) {
    if (h.empty()) return HMS_OK;
    HIPTRY(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return HMS_OK;
}

hms_status load_plan(hms::HostPlan&& plan, void* stream, hms_cnf** out) {
    int dev = -1;
    hms_status st = current_gfx950(dev);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    hms_cnf* C = new (std::nothrow) hms_cnf();
    if (!C) return fail(HMS_ERR_NOMEM, "host allocation failed");
    C->plan = std::move(plan);
    C->device = dev;
    const hms::HostPlan& P = C->plan;
    Layout L;
    size_t o_ct = L.add(P.c_tile.size() * sizeof(hms::TileDesc));
    size_t o_ce = L.add(P.c_ent.size() * 4);
    size_t o_vt = L.add(P.v_tile.size() * sizeof(hms::TileDesc));
    size_t o_ve = L.add(P.v_ent.size() * 4);
    size_t o_sf = L.add(P.seg_first.size() * 4);
    size_t o_vo = L.add(P.var_old.size() * 4);
    size_t o_w = L.add(P.c_w.size() * 8);
    const bool slots = P.slot_ok && !P.c_ent.empty();
    size_t o_cs = L.add(slots ? P.c_ent.size() * 4 : 0);
    void* base = nullptr;
    hipError_t e = hipMalloc(&base, std::max<size_t>(L.off, 256));
    if (e != hipSuccess) {
        delete C;
        return fail(e == hipErrorOutOfMemory ? HMS_ERR_NOMEM : HMS_ERR_DEVICE,
                    std::string("hipMalloc of the instance structure: ") + hipGetErrorString(e));
    }
    char* b = (char*)base;
    C->arena = base;
    C->c_tile = (hms::TileDesc*)(b + o_ct);
    C->c_ent = (uint32_t*)(b + o_ce);
    C->v_tile = (hms::TileDesc*)(b + o_vt);
    C->v_ent = (uint32_t*)(b + o_ve);
    C->seg_first = (int32_t*)(b + o_sf);
    C->var_old = (int32_t*)(b + o_vo);
    C->c_w = P.c_w.empty() ? nullptr : (int64_t*)(b + o_w);
    C->c_slot = slots ? (uint32_t*)(b + o_cs) : nullptr;
    C->struct_bytes = (int64_t)L.off;
    hms_status r = HMS_OK;
    if (!r) r = upload(P.c_tile, C->c_tile, s);
    if (!r) r = upload(P.c_ent, C->c_ent, s);
    if (!r) r = upload(P.v_tile, C->v_tile, s);
    if (!r) r = upload(P.v_ent, C->v_ent, s);
    if (!r) r = upload(P.seg_first, C->seg_first, s);
    if (!r) r = upload(P.var_old, C->var_old, s);
    if (!r) r = upload(P.c_w, C->c_w, s);
    if (!r && slots) {
        // the occurrence map of the slot schedules, built from the uploaded sides
        hms::SlotArgs sa{};
        sa.c_tile = C->c_tile;
        sa.c_ent = C->c_ent;
        sa.v_tile = C->v_tile;
        sa.v_ent = C->v_ent;
        sa.seg_first = C->seg_first;
        sa.n_heavy = P.n_heavy;
        sa.seg_rows = P.seg_rows;
        sa.seg_tiles = P.seg_tiles;
        sa.v_tiles = P.v_tiles;
        sa.vpad = (uint32_t)P.a_zero_row();
        sa.c_slot = C->c_slot;
        sa.c_ent_n = (int64_t)P.c_ent.size();
        e = hms::launch_build_slots(sa, s);
        if (e != hipSuccess) r = fail(HMS_ERR_DEVICE, std::string("occurrence map: ") + hipGetErrorString(e));
    }
    if (!r) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) r = fail(HMS_ERR_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    if (r) {
        (void)hipStreamSynchronize(s);  // copies already queued read the plan
        hms_free_cnf(C);
        return r;
    }
    *out = C;
    return HMS_OK;
}

}  // namespace

extern "C" {

const char* hms_last_error(void) { return g_err.c_str(); }

const char* hms_version(void) { return "hipmsat 0.1 (gfx950)"; }

hms_status hms_load_wcnf(int32_t n_vars, const int32_t* lits, int64_t n_lits, const int64_t* weights, void* stream,
                         hms_cnf** out) {
    g_err.clear();
    if (!out) return fail(HMS_ERR_ARG, "null output pointer");
    *out = nullptr;
    hms::HostPlan plan;
    std::string err;
    int32_t rc = hms::build_plan(n_vars, lits, n_lits, weights, plan, err);
    if (rc) return fail(rc, err);
    return load_plan(std::move(plan), stream, out);
}

hms_status hms_load_cnf(int32_t n_vars, const int32_t* lits, int64_t n_lits, void* stream, hms_cnf** out) {
    return hms_load_wcnf(n_vars, lits, n_lits, nullptr, stream, out);
}

hms_status hms_load_cnf_dimacs(const char* path, void* stream, hms_cnf** out) {
    g_err.clear();
    if (!out || !path) return fail(HMS_ERR_ARG, "null argument");
    *out = nullptr;
    int32_t n = 0;
    std::vector<int32_t> lits;
    std::vector<int64_t> weights;
    std::string err;
    int32_t rc = hms::read_dimacs(path, n, lits, weights, err);
    if (rc) return fail(rc, err);
    return hms_load_wcnf(n, lits.data(), (int64_t)lits.size(), weights.empty() ? nullptr : weights.data(), stream,
                         out);
}

void hms_free_cnf(hms_cnf* cnf) {
    if (!cnf) return;
    if (cnf->arena) {
        DeviceGuard g(cnf->device);
        (void)hipFree(cnf->arena);
    }
    delete cnf;
}

hms_status hms_cnf_info_get(const hms_cnf* cnf, hms_cnf_info* out) {
    g_err.clear();
    if (check_cnf(cnf) || !out) return fail(HMS_ERR_ARG, "null argument");
    const hms::HostPlan& P = cnf->plan;
    out->n_vars = P.n;
    out->n_clauses = P.m;
    out->n_lits = P.lits_in;
    out->nnz = P.nnz;
    out->n_empty = P.m_empty;
    out->n_taut = P.m_taut;
    out->n_active = P.n_act;
    out->n_heavy = P.n_heavy;
    out->struct_bytes = cnf->struct_bytes;
    // x, m, v, t, best bytes, a, heavy partials per restart
    out->state_bytes_r1 = (int64_t)(P.n + 1) * 16 + P.n + (int64_t)P.a_rows() * 4 + (int64_t)P.seg_rows * 8;
    out->weighted = P.weighted ? 1 : 0;
    out->total_weight = P.w_total;
    out->plan_threads = P.build_threads;
    out->slot_bytes = cnf->c_slot ? (int64_t)P.v_ent.size() * 4 : 0;
    return HMS_OK;
}

void hms_solve_params_default(hms_solve_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->steps = 1000;
    p->restarts = 1;
    p->eval_every = 1;
    p->optimizer = HMS_ADAM;
    p->seed = 0;
    p->lr = 1e-4f;
    p->beta1 = 0.9f;
    p->beta2 = 0.999f;
    p->eps = 1e-8f;
    p->loss_mode = HMS_LOSS_UNSAT;
    p->schedule = 0;
    p->use_graph = 1;
    p->autotune = 1;
    p->time_limit_s = 0.0;
    p->x0 = nullptr;
    p->stream = nullptr;
}

}  // extern "C"

namespace {

// Validated set-up shared by hms_solve and hms_time_kernels: state arena,
// initial point, launch arguments.
struct SolveSetup {
    Arena A;
    State S{};
    Shape sh{};
    Launch L{};
    int32_t step0 = 0;  // iterations taken before this call (a resumed solve)
};

// A state a solve resumes from or hands back: every array it needs is given.
hms_status check_state(const hms_cnf* cnf, const hms_solve_params* p, const hms_solve_state* st, const char* what) {
    const bool has_n = cnf->plan.n > 0;
    const bool adam = p->optimizer == HMS_ADAM;
    if ((has_n && (!st->x || !st->best_assignment)) || !st->best || !st->best_step ||
        (adam && has_n && (!st->m || !st->v)))
        return fail(HMS_ERR_ARG, std::string(what) + ": a required state array is null");
    return HMS_OK;
}

static_assert(sizeof(hms::TracePoint) == sizeof(hms_trace_point), "trace record layout");

// Rows of a solve's trajectory: one per count, at t % K == 0 for t in
// [s0, t_end) and at t_end, the count at t in row ceil(t / K) - ceil(s0 / K).
int64_t trace_rows(int32_t s0, int32_t t_end, int32_t K) {
    return ((int64_t)t_end + K - 1) / K - ((int64_t)s0 + K - 1) / K + 1;
}

// Copy a device trajectory ring into res->trace, oldest row first
// (synchronises s).
hms_status read_trace(const hms::TracePoint* ring, int32_t R, int32_t K, int32_t s0, int32_t t_end, hipStream_t s,
                      hms_solve_result* res) {
    const int64_t total = trace_rows(s0, t_end, K);
    const int64_t cap = res->trace_cap;
    const int64_t stored = std::min(total, cap);
    std::vector<hms::TracePoint> h((size_t)(cap * R));  // before the guard: a queued copy writes it
    SyncOnExit copy_done{s};
    HIPTRY(hipMemcpyAsync(h.data(), ring, h.size() * sizeof(hms::TracePoint), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    for (int64_t j = 0; j < stored; ++j) {
        const int64_t row = (total - stored + j) % cap;
        std::memcpy(res->trace + j * R, h.data() + row * R, (size_t)R * sizeof(hms::TracePoint));
    }
    res->trace_len = (int32_t)stored;
    return HMS_OK;
}

// Checks of hms_solve's resume input and state output.
hms_status check_resume(const hms_cnf* cnf, const hms_solve_params* p, const hms_solve_result* res) {
    if (res->trace && (res->trace_cap < 1 || (int64_t)res->trace_cap * std::max(p->restarts, 1) > (1 << 26)))
        return fail(HMS_ERR_ARG, "trace needs 1 <= trace_cap and trace_cap * restarts <= 2^26");
    if (p->resume) {
        if (p->x0) return fail(HMS_ERR_ARG, "x0 and resume are both given");
        hms_status rc = check_state(cnf, p, p->resume, "resume");
        if (rc) return rc;
        if (p->resume->step < 0 || p->steps < 0 || p->resume->step > INT32_MAX - p->steps)
            return fail(HMS_ERR_ARG, "resume step out of range (0 <= step, step + steps < 2^31)");
    }
    if (res->state) return check_state(cnf, p, res->state, "state output");
    return HMS_OK;
}

hms_status setup_solve(const hms_cnf* cnf, const hms_solve_params* p, SolveSetup& Z) {
    if (check_cnf(cnf) || !p) return fail(HMS_ERR_ARG, "null argument");
    const int32_t R = p->restarts, T = p->steps, K = p->eval_every;
    if (R < 1 || T < 0 || K < 1) return fail(HMS_ERR_ARG, "restarts >= 1, steps >= 0 and eval_every >= 1 required");
    if (p->optimizer != HMS_ADAM && p->optimizer != HMS_SGD) return fail(HMS_ERR_ARG, "unknown optimizer");
    if (p->loss_mode != HMS_LOSS_UNSAT && p->loss_mode != HMS_LOSS_ALL) return fail(HMS_ERR_ARG, "unknown loss mode");
    if (!std::isfinite(p->lr) || !std::isfinite(p->beta1) || !std::isfinite(p->beta2) || !std::isfinite(p->eps))
        return fail(HMS_ERR_ARG, "non-finite optimizer parameter");
    const hms::HostPlan& P = cnf->plan;
    // state elements per array; the element-wise kernels' grids (256 per workgroup) stay within 2^31
    if ((int64_t)(P.n + 1) * R > ((int64_t)1 << 38)) return fail(HMS_ERR_TOO_LARGE, "state too large");
    hipStream_t s = (hipStream_t)p->stream;
    hms_status rc = make_shape(P, R, p->schedule, p->loss_mode, Z.sh);
    if (rc) return rc;
    const bool adam = p->optimizer == HMS_ADAM;
    Layout lay;
    size_t off[kOffN];
    layout_state(P, Z.sh, adam, false, true, lay, off);
    Z.A.s = s;
    HIPTRY(hipMallocAsync((void**)&Z.A.base, lay.off, s));
    Z.S = bind_state(Z.A, off, adam, false, true);
    hms::InitArgs ia = make_init(cnf, Z.sh, Z.S);
    ia.x0 = p->x0;
    ia.seed = p->seed;
    if (const hms_solve_state* rs = p->resume) {
        // continue from the caller's state: the best so far goes into the
        // tracking arrays before the init kernel, which then keeps it
        SyncOnExit up{s};  // the host arrays are read by queued copies
        HIPTRY(hipMemcpyAsync(Z.S.best, rs->best, (size_t)R * 8, hipMemcpyHostToDevice, s));
        HIPTRY(hipMemcpyAsync(Z.S.best_step, rs->best_step, (size_t)R * 4, hipMemcpyHostToDevice, s));
        ia.x0 = rs->x;
        ia.m0 = adam ? rs->m : nullptr;
        ia.v0 = adam ? rs->v : nullptr;
        ia.best_a0 = rs->best_assignment;
        ia.step0 = rs->step;
        ia.keep_best = 1;
        Z.step0 = rs->step;
    }
    HIPTRY(hms::launch_init(ia, s));
    Z.L = make_launch(cnf, Z.sh, Z.S, adam ? hms::kAdam : hms::kSgd, p->loss_mode, p->lr, p->beta1, p->beta2,
                      p->eps);
    return HMS_OK;
}

struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Events() {
        for (auto x : e)
            if (x) (void)hipEventDestroy(x);
    }
};


bool resident_ok(const hms_cnf* cnf, const hms_solve_params* p);
bool resident_preferred(const hms_cnf* cnf, const hms_solve_params* p);
hms_status time_resident(const hms_cnf* cnf, const hms_solve_params* p0, int32_t iters, double& ms);
constexpr int32_t kResidentId = 0xff;
constexpr int64_t kResidentNnz = 1 << 15;  // largest instance the untimed choice sends to the resident solver

uint64_t tune_key(const hms_solve_params* p) {
    return (uint64_t)(uint32_t)p->restarts | ((uint64_t)(uint32_t)p->optimizer << 32) |
           ((uint64_t)(uint32_t)p->loss_mode << 40);
}

int ilog2(int64_t v) {
    int k = 0;
    while (v > 1) {
        v >>= 1;
        ++k;
    }
    return k;
}

// Process-wide cache by size class (restarts, optimizer, loss mode, log2 nnz,
// log2 n): a new instance of a size already tuned reuses that choice.
std::mutex g_tune_mu;
std::map<uint64_t, int32_t> g_tuned;

uint64_t class_key(const hms_cnf* cnf, const hms_solve_params* p) {
    return tune_key(p) ^ ((uint64_t)ilog2(cnf->plan.nnz + 1) << 48) ^ ((uint64_t)ilog2(cnf->plan.n + 1) << 56);
}

// Every (schedule, rows per unit) pair that can run R restarts.
std::vector<int32_t> tune_candidates(int32_t R, int loss_mode) {
    std::vector<int32_t> out;
    for (int idx = 1; idx <= hms::kNumSchedules; ++idx) {
        const hms::Schedule& c = hms::kSchedules[idx];
        if (R % c.V) continue;
        if (c.mask && loss_mode != HMS_LOSS_UNSAT) continue;
        if (c.slot && (R != 1 || loss_mode != HMS_LOSS_UNSAT)) continue;
        if (c.P * c.V > 4 * std::max(R, 1)) continue;  // mostly idle lanes
        if (c.nt > 1 && R > 4) continue;  // many restarts already give every wavefront enough reads
        const int per = (64 / c.P) * c.UR;
        for (int U = per; U <= 64; U *= 2) {
            if (64 % U || (c.mask && U < 32)) continue;
            out.push_back(idx | (U << 8));
        }
    }
    return out;
}

// Average device time of one step under schedule `code`, counting every
// eval_every steps as a solve does (the counting passes weigh heavily when
// eval_every is small).
hms_status time_steps(const hms_cnf* cnf, const hms_solve_params* p0, int32_t code, int32_t iters, double& ms) {
    hms_solve_params p = *p0;
    p.schedule = code;
    p.x0 = nullptr;
    p.resume = nullptr;
    SolveSetup Z;
    hms_status rc = setup_solve(cnf, &p, Z);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)p.stream;
    Events E;
    for (int i = 0; i < 2; ++i) HIPTRY(hipEventCreate(&E.e[i]));
    const int32_t K = std::max(p.eval_every, 1);
    iters = std::max(iters, std::min(K, 64));  // at least one counting step when K is small
    HIPTRY(enqueue_step(Z.L, true, s));
    if (p.use_graph) {
        // as a solve replays its steps: from a captured graph, so the launch
        // gaps are the graph's, not the host's
        struct G {
            hipStream_t cs = nullptr;
            hipGraph_t g = nullptr;
            hipGraphExec_t x = nullptr;
            hipStream_t user = nullptr;
            ~G() {
                if (user) (void)hipStreamSynchronize(user);
                if (x) (void)hipGraphExecDestroy(x);
                if (g) (void)hipGraphDestroy(g);
                if (cs) (void)hipStreamDestroy(cs);
            }
        } gr;
        gr.user = s;
        HIPTRY(hipStreamCreateWithFlags(&gr.cs, hipStreamNonBlocking));
        HIPTRY(hipStreamBeginCapture(gr.cs, hipStreamCaptureModeRelaxed));
        hipError_t ce = hipSuccess;
        for (int32_t i = 0; i < iters && ce == hipSuccess; ++i) ce = enqueue_step(Z.L, i % K == 0, gr.cs);
        hipError_t ee = hipStreamEndCapture(gr.cs, &gr.g);
        if (ce != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(ce));
        if (ee != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(ee));
        HIPTRY(hipGraphInstantiate(&gr.x, gr.g, nullptr, nullptr, 0));
        HIPTRY(hipGraphLaunch(gr.x, s));  // warm-up
        HIPTRY(hipEventRecord(E.e[0], s));
        HIPTRY(hipGraphLaunch(gr.x, s));
        HIPTRY(hipEventRecord(E.e[1], s));
        HIPTRY(hipStreamSynchronize(s));
        float t1 = 0;
        HIPTRY(hipEventElapsedTime(&t1, E.e[0], E.e[1]));
        // short steps: replay until about 2 ms are timed, so launch jitter
        // does not decide between near-equal schedules
        const int reps = t1 > 0 ? std::min(64, (int)std::ceil(2.0 / t1)) : 1;
        if (reps > 1) {
            HIPTRY(hipEventRecord(E.e[0], s));
            for (int k = 0; k < reps; ++k) HIPTRY(hipGraphLaunch(gr.x, s));
            HIPTRY(hipEventRecord(E.e[1], s));
            iters *= reps;
        }
    } else {
        HIPTRY(hipEventRecord(E.e[0], s));
        for (int32_t i = 0; i < iters; ++i) HIPTRY(enqueue_step(Z.L, i % K == 0, s));
        HIPTRY(hipEventRecord(E.e[1], s));
    }
    HIPTRY(hipStreamSynchronize(s));
    float t = 0;
    HIPTRY(hipEventElapsedTime(&t, E.e[0], E.e[1]));
    ms = t / iters;
    return HMS_OK;
}

// Average device time of the forward pass alone and of the backward pass
// (with the heavy-row combine) alone under schedule `code`.
hms_status time_split(const hms_cnf* cnf, const hms_solve_params* p0, int32_t code, int32_t iters, double& fwd_ms,
                      double& bwd_ms) {
    hms_solve_params p = *p0;
    p.schedule = code;
    p.x0 = nullptr;
    p.resume = nullptr;
    SolveSetup Z;
    hms_status rc = setup_solve(cnf, &p, Z);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)p.stream;
    const Launch& L = Z.L;
    Events E;
    for (int i = 0; i < 3; ++i) HIPTRY(hipEventCreate(&E.e[i]));
    HIPTRY(enqueue_step(L, false, s));
    HIPTRY(hipEventRecord(E.e[0], s));
    for (int32_t i = 0; i < iters; ++i) HIPTRY(hms::launch_fwd(Z.sh.sched, false, L.fa, Z.sh.fwd_blocks, s));
    HIPTRY(hipEventRecord(E.e[1], s));
    for (int32_t i = 0; i < iters; ++i) {
        HIPTRY(hms::launch_bwd(Z.sh.sched, L.opt, L.ba, Z.sh.bwd_blocks, s));
        HIPTRY(hms::launch_combine(L.opt, L.ba, s));
    }
    HIPTRY(hipEventRecord(E.e[2], s));
    HIPTRY(hipStreamSynchronize(s));
    float a = 0, b = 0;
    HIPTRY(hipEventElapsedTime(&a, E.e[0], E.e[1]));
    HIPTRY(hipEventElapsedTime(&b, E.e[1], E.e[2]));
    fwd_ms = a / iters;
    bwd_ms = b / iters;
    return HMS_OK;
}

// Autotuner: for every table entry, the forward and the backward pass each
// take their fastest rows per unit (timed apart), then whole steps of each
// entry's pair are timed against each other (and the resident solver).
hms_status tune(const hms_cnf* cnf, const hms_solve_params* p, int32_t iters, int32_t& best, double& best_ms) {
    best = 0;
    best_ms = 1e300;
    struct Pick {
        double f = 1e300, b = 1e300;
        int Uf = 0, Ub = 0;
    };
    std::map<int, Pick> picks;
    for (int32_t code : tune_candidates(p->restarts, p->loss_mode)) {
        double f = 0, b = 0;
        hms_status rc = time_split(cnf, p, code, iters, f, b);
        if (rc) return rc;
        Pick& k = picks[code & 0xff];
        const int U = (code >> 8) & 0xff;
        if (f < k.f) {
            k.f = f;
            k.Uf = U;
        }
        if (b < k.b) {
            k.b = b;
            k.Ub = U;
        }
    }
    std::vector<int32_t> cands;
    for (auto& kv : picks) cands.push_back(kv.first | (kv.second.Uf << 8) | (kv.second.Ub << 16));
    if (resident_ok(cnf, p)) cands.push_back(kResidentId);
    auto time_code = [&](int32_t code, double& ms) {
        return code == kResidentId ? time_resident(cnf, p, iters, ms) : time_steps(cnf, p, code, iters, ms);
    };
    std::vector<std::pair<double, int32_t>> timed;
    for (int32_t code : cands) {
        double ms = 0;
        hms_status rc = time_code(code, ms);
        if (rc) return rc;
        timed.emplace_back(ms, code);
    }
    // the three fastest, and the entry the untimed rule would take, are
    // timed twice more and keep their best time, so that one noisy
    // measurement does not decide between near-equal choices
    std::sort(timed.begin(), timed.end());
    const int untimed = auto_schedule(p->restarts, p->loss_mode, cnf->plan.nnz, cnf->plan.n_act);
    for (size_t k = 0; k < timed.size(); ++k) {
        if (k >= 3 && (timed[k].second == kResidentId || (timed[k].second & 0xff) != untimed)) continue;
        for (int rep = 0; rep < 2; ++rep) {
            double ms = 0;
            hms_status rc = time_code(timed[k].second, ms);
            if (rc) return rc;
            timed[k].first = std::min(timed[k].first, ms);
        }
    }
    for (const auto& tc : timed)
        if (tc.first < best_ms) {
            best_ms = tc.first;
            best = tc.second;
        }
    if (best != kResidentId && ((best >> 16) & 0xff) == ((best >> 8) & 0xff)) best &= 0xffff;  // canonical id
    {
        std::lock_guard<std::mutex> lk(cnf->tune_mu);
        cnf->tuned[tune_key(p)] = best;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[class_key(cnf, p)] = best;
    return HMS_OK;
}

// Schedule to run when the caller asked for the automatic choice.
hms_status resolve_schedule(const hms_cnf* cnf, const hms_solve_params* p, int32_t& code) {
    code = p->schedule;
    if (code != 0) return HMS_OK;
    {
        std::lock_guard<std::mutex> lk(cnf->tune_mu);
        auto it = cnf->tuned.find(tune_key(p));
        // the resident solver cannot honour a time limit or a cancel flag:
        // a solve that asks for one takes the tiled choice below instead
        if (it != cnf->tuned.end() && (it->second != kResidentId || resident_ok(cnf, p))) {
            code = it->second;
            return HMS_OK;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(class_key(cnf, p));
        if (it != g_tuned.end() && (it->second != kResidentId || resident_ok(cnf, p))) {
            code = it->second;
            return HMS_OK;
        }
    }
    if (!p->autotune || (double)cnf->plan.nnz * p->restarts < (double)(1 << 18)) {
        if (resident_preferred(cnf, p)) code = kResidentId;  // small: launch latency dominates
        return HMS_OK;
    }
    double ms = 0;
    return tune(cnf, p, 6, code, ms);
}

// ---- resident path (one workgroup per restart, state in LDS) ---------------
constexpr int32_t kResident = kResidentId;  // schedule id of the resident solver

size_t lds_limit(int dev) {
    static std::atomic<size_t> cached[64] = {};  // per device; solves on several threads may fill it at once
    if (dev >= 0 && dev < 64) {
        const size_t c = cached[dev].load(std::memory_order_relaxed);
        if (c) return c;
    }
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
    const size_t stat = hms::small_static_lds();  // the kernel's own LDS comes on top
    const size_t lim = (size_t)v > stat ? (size_t)v - stat : 0;
    if (dev >= 0 && dev < 64) cached[dev].store(lim, std::memory_order_relaxed);
    return lim;
}

// Without timing, the resident solver is taken for instances of at most
// kResidentNnz nonzeros (twice that when every step is counted): one
// workgroup then costs about 1.4 us + 0.2 ns per nonzero per step, the tiled
// launches 7-8 us per step (about 14 with a count every step).
bool resident_preferred(const hms_cnf* cnf, const hms_solve_params* p) {
    const int64_t lim = p->eval_every <= 1 ? 2 * kResidentNnz : kResidentNnz;
    return cnf->plan.nnz <= lim && resident_ok(cnf, p);
}

bool resident_ok(const hms_cnf* cnf, const hms_solve_params* p) {
    const hms::HostPlan& P = cnf->plan;
    // the resident solver runs the whole loop in one launch: no time limit or cancel flag can stop it
    return P.n_heavy_wide == 0 && p->time_limit_s <= 0 && p->cancel == nullptr &&
           hms::small_lds_bytes(P) <= lds_limit(cnf->device);
}

// Rows a resident workgroup walks per phase: the larger plan side.
int32_t resident_rows(const hms_cnf* cnf) {
    return std::max(cnf->plan.c_tiles, cnf->plan.v_tiles) * hms::kTile;
}

// LDS of one resident workgroup for this instance: state plus the staged plan.
size_t resident_lds(const hms_cnf* cnf) {
    return hms::small_lds_total(cnf->plan, lds_limit(cnf->device), nullptr);
}

hms::SmallDesc make_desc(const hms_cnf* cnf, const hms_solve_params* p) {
    const hms::HostPlan& P = cnf->plan;
    hms::SmallDesc D{};
    D.c_tile = cnf->c_tile;
    D.c_ent = cnf->c_ent;
    D.v_tile = cnf->v_tile;
    D.v_ent = cnf->v_ent;
    D.seg_first = cnf->seg_first;
    D.var_old = cnf->var_old;
    D.n = P.n;
    D.m = P.m;
    D.n_act = P.n_act;
    D.n_heavy = P.n_heavy;
    D.c_tiles = P.c_tiles;
    D.v_tiles = P.v_tiles;
    D.seg_tiles = P.seg_tiles;
    D.seg_rows = P.seg_rows;
    D.w_empty = P.w_empty;
    D.best0 = P.w_total;
    D.c_w = cnf->c_w;
    D.c_ent_len = (int32_t)P.c_ent.size();
    D.v_ent_len = (int32_t)P.v_ent.size();
    hms::small_lds_total(P, lds_limit(cnf->device), &D.stage);
    D.R = p->restarts;
    D.T = p->steps;
    D.K = p->eval_every;
    D.opt = p->optimizer == HMS_SGD ? hms::kSgd : hms::kAdam;
    D.all_mode = p->loss_mode == HMS_LOSS_ALL;
    D.two_over_m = P.m > 0 ? (float)(2.0 / (double)P.m) : 0.0f;
    D.inv_m = P.m > 0 ? 1.0 / (double)P.m : 0.0;
    D.lr = p->lr;
    D.b1 = p->beta1;
    D.b2 = p->beta2;
    D.eps = p->eps;
    D.omb1 = 1.0f - p->beta1;
    D.omb2 = 1.0f - p->beta2;
    D.lr_d = (double)p->lr;
    D.b1_d = (double)p->beta1;
    D.b2_d = (double)p->beta2;
    D.seed = p->seed;
    D.x0 = p->x0;
    return D;
}

// Device outputs of one resident instance, carved from an arena.
struct SmallOut {
    size_t o_best_a, o_best, o_step, o_loss;
};

SmallOut layout_small_out(const hms::HostPlan& P, int32_t R, Layout& L) {
    SmallOut o;
    o.o_best_a = L.add((size_t)std::max(P.n, 1) * R);
    o.o_best = L.add((size_t)R * 8);
    o.o_step = L.add((size_t)R * 4);
    o.o_loss = L.add((size_t)R * 8);
    return o;
}

hms_status solve_resident(const hms_cnf* cnf, const hms_solve_params* p, hms_solve_result* res) {
    const hms::HostPlan& P = cnf->plan;
    const int32_t R = p->restarts;
    const bool adam = p->optimizer == HMS_ADAM;
    hipStream_t s = (hipStream_t)p->stream;
    const hms_solve_state* rs = p->resume;
    hms_solve_state* so = res->state;
    // host destinations of the copies below: declared before the guard that
    // waits for the stream, so an early return cannot free them under a copy
    std::vector<int64_t> best(R);
    std::vector<int32_t> bstep(R);
    std::vector<double> closs(R);
    Layout lay;
    const size_t o_desc = lay.add(sizeof(hms::SmallDesc));
    SmallOut so_l = layout_small_out(P, R, lay);
    const size_t o_trace = res->trace ? lay.add((size_t)res->trace_cap * R * sizeof(hms::TracePoint)) : 0;
    Arena A;
    A.s = s;
    HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
    hms::SmallDesc D = make_desc(cnf, p);
    if (res->trace) {
        D.trace = A.at<hms::TracePoint>(o_trace);
        D.trace_cap = res->trace_cap;
    }
    D.block0 = 0;
    D.best_a = A.at<uint8_t>(so_l.o_best_a);
    D.best = A.at<int64_t>(so_l.o_best);
    D.best_step = A.at<int32_t>(so_l.o_step);
    D.final_loss = A.at<double>(so_l.o_loss);
    D.x_final = res->x_final ? res->x_final : (so ? so->x : nullptr);
    if (so && adam) {
        D.m_final = so->m;
        D.v_final = so->v;
    }
    if (rs) {
        D.x0 = rs->x;
        D.m0 = adam ? rs->m : nullptr;
        D.v0 = adam ? rs->v : nullptr;
        D.step0 = rs->step;
        D.resume = 1;
    }
    Events E;
    for (int i = 0; i < 2; ++i) HIPTRY(hipEventCreate(&E.e[i]));
    SyncOnExit d_done{s};
    HIPTRY(hipMemcpyAsync(A.base + o_desc, &D, sizeof(D), hipMemcpyHostToDevice, s));
    if (rs) {
        // the resumed best enters through the output arrays the kernel updates
        HIPTRY(hipMemcpyAsync(D.best, rs->best, (size_t)R * 8, hipMemcpyHostToDevice, s));
        HIPTRY(hipMemcpyAsync(D.best_step, rs->best_step, (size_t)R * 4, hipMemcpyHostToDevice, s));
        if (P.n > 0)
            HIPTRY(hipMemcpyAsync(D.best_a, rs->best_assignment, (size_t)R * P.n, hipMemcpyDeviceToDevice, s));
    }
    HIPTRY(hipEventRecord(E.e[0], s));
    HIPTRY(hms::launch_small(A.at<hms::SmallDesc>(o_desc), 1, R, resident_lds(cnf), lds_limit(cnf->device), D.stage,
                             resident_rows(cnf), hms::small_reg_ok(cnf->plan, resident_rows(cnf)), s));
    HIPTRY(hipEventRecord(E.e[1], s));
    HIPTRY(hipMemcpyAsync(best.data(), D.best, R * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(bstep.data(), D.best_step, R * 4, hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(closs.data(), D.final_loss, R * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    int32_t br = 0;
    for (int32_t r = 1; r < R; ++r)
        if (best[r] < best[br]) br = r;
    if (res->best_assignment && P.n > 0)
        HIPTRY(hipMemcpyAsync(res->best_assignment, D.best_a + (size_t)br * P.n, P.n, hipMemcpyDeviceToHost, s));
    if (so && P.n > 0) {
        if (res->x_final && so->x != res->x_final)
            HIPTRY(hipMemcpyAsync(so->x, res->x_final, (size_t)P.n * R * 4, hipMemcpyDeviceToDevice, s));
        HIPTRY(hipMemcpyAsync(so->best_assignment, D.best_a, (size_t)R * P.n, hipMemcpyDeviceToDevice, s));
    }
    HIPTRY(hipStreamSynchronize(s));
    float ms = 0;
    HIPTRY(hipEventElapsedTime(&ms, E.e[0], E.e[1]));
    res->best_cost = best[br];
    res->best_restart = br;
    res->best_step = bstep[br];
    res->steps_done = p->steps;
    res->schedule = kResident;
    res->final_loss = closs[br];
    res->device_ms = ms;
    if (res->restart_best) std::memcpy(res->restart_best, best.data(), R * 8);
    if (res->restart_step) std::memcpy(res->restart_step, bstep.data(), R * 4);
    if (res->restart_loss) std::memcpy(res->restart_loss, closs.data(), R * 8);
    if (so) {
        std::memcpy(so->best, best.data(), R * 8);
        std::memcpy(so->best_step, bstep.data(), R * 4);
        so->step = (rs ? rs->step : 0) + p->steps;
    }
    if (res->trace) {
        const int32_t s0 = rs ? rs->step : 0;
        if (hms_status rt = read_trace(D.trace, R, p->eval_every, s0, s0 + p->steps, s, res)) return rt;
    }
    for (int32_t r = 0; r < R; ++r)
        if (!std::isfinite(closs[r])) return fail(HMS_ERR_NONFINITE, "the loss at the final iterate is not finite");
    return HMS_OK;
}

// Device time per step of a short resident solve.
// Device time per step of the resident solver: the difference between a
// short and a three times longer solve, so the launch and set-up cost (paid
// once per solve) does not count as per-step time.
hms_status time_resident(const hms_cnf* cnf, const hms_solve_params* p0, int32_t iters, double& ms) {
    hms_solve_params p = *p0;
    p.eval_every = std::max(p0->eval_every, 1);
    p.x0 = nullptr;
    p.resume = nullptr;
    const int32_t S = std::max(iters, 16) * 4;
    double t[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {  // the first solve only warms the device up
        p.steps = k == 2 ? 3 * S : S;
        hms_solve_result r{};
        hms_status rc = solve_resident(cnf, &p, &r);
        if (rc) return rc;
        t[k] = r.device_ms;
    }
    ms = std::max(t[2] - t[1], 0.0) / (2.0 * S);
    return HMS_OK;
}

// The count at x_T (always taken) and the snapshot of the best assignment.
hipError_t count_final(const hms_cnf* cnf, const SolveSetup& Z, hipStream_t s) {
    const Shape& sh = Z.sh;
    hipError_t e = hms::launch_fwd(sh.sched, true, Z.L.fa, sh.fwd_blocks, s);
    if (e == hipSuccess) e = hms::launch_reduce(Z.L.ra, s);
    if (e == hipSuccess) e = hms::launch_snapshot(cnf->plan.n_act, sh.B, Z.S.x, Z.S.improved, Z.S.best_a, s);
    return e;
}

// Read a finished solve's outcome into `res` (synchronises s), and the state
// after its last step into res->state when asked.
hms_status read_result(const hms_cnf* cnf, const SolveSetup& Z, int32_t done, float ms, hipStream_t s,
                       hms_solve_result* res) {
    const hms::HostPlan& P = cnf->plan;
    const Shape& sh = Z.sh;
    const State& S = Z.S;
    const int32_t R = sh.B.R;
    hms_solve_state* so = res->state;
    // host destinations of the copies below, declared before the guard that
    // waits for the stream: an early return cannot free them under a copy
    std::vector<int64_t> best(R);
    std::vector<int32_t> bstep(R);
    std::vector<double> closs(R);
    SyncOnExit copies_done{s};
    HIPTRY(hipMemcpyAsync(best.data(), S.best, R * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(bstep.data(), S.best_step, R * 4, hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(closs.data(), S.cur_loss, R * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    int32_t br = 0;
    for (int32_t r = 1; r < R; ++r)
        if (best[r] < best[br]) br = r;
    if (res->best_assignment && P.n > 0) {
        HIPTRY(hms::launch_extract(P.n, sh.B, br, cnf->var_old, S.best_a, S.out_assign, s));
        HIPTRY(hipMemcpyAsync(res->best_assignment, S.out_assign, P.n, hipMemcpyDeviceToHost, s));
    }
    if (res->x_final) HIPTRY(hms::launch_scatter(P.n, P.n, sh.B, cnf->var_old, S.x, res->x_final, s));
    if (so) {
        HIPTRY(hms::launch_scatter(P.n, P.n, sh.B, cnf->var_old, S.x, so->x, s));
        if (S.m) {
            HIPTRY(hms::launch_scatter(P.n, P.n, sh.B, cnf->var_old, S.m, so->m, s));
            HIPTRY(hms::launch_scatter(P.n, P.n, sh.B, cnf->var_old, S.v, so->v, s));
        }
        HIPTRY(hms::launch_scatter_bytes(P.n, sh.B, cnf->var_old, S.best_a, so->best_assignment, s));
    }
    HIPTRY(hipStreamSynchronize(s));
    res->best_cost = best[br];
    res->best_restart = br;
    res->best_step = bstep[br];
    res->steps_done = done;
    res->schedule = sh.code;
    res->final_loss = closs[br];
    res->device_ms = ms;
    if (res->restart_best) std::memcpy(res->restart_best, best.data(), R * 8);
    if (res->restart_step) std::memcpy(res->restart_step, bstep.data(), R * 4);
    if (res->restart_loss) std::memcpy(res->restart_loss, closs.data(), R * 8);
    if (so) {
        std::memcpy(so->best, best.data(), R * 8);
        std::memcpy(so->best_step, bstep.data(), R * 4);
        so->step = Z.step0 + done;
    }
    for (int32_t r = 0; r < R; ++r)
        if (!std::isfinite(closs[r])) return fail(HMS_ERR_NONFINITE, "the loss at the final iterate is not finite");
    return HMS_OK;
}

// Steps of the graph body: a multiple of K starting at a multiple of K.
int32_t graph_body(int32_t K) { return K * std::max(1, (32 + K - 1) / K); }

// Tiled instances of a batch that share restarts, steps, counting period,
// optimizer and loss mode: every step is one launch per kernel for all of
// them (each workgroup finds its instance from the running block counts),
// replayed as a HIP graph.  Each instance's arguments are those of its own
// solve, so its result is bitwise the one it gets alone.
hms_status solve_tiled_group(const hms_cnf* const* cnfs, const hms_solve_params* params, const int32_t* idx,
                             int32_t cnt, int32_t code, hipStream_t s, hms_solve_result* results,
                             hms_status* statuses) {
    std::vector<std::unique_ptr<SolveSetup>> Z(cnt);
    for (int32_t k = 0; k < cnt; ++k) {
        hms_solve_params p = params[idx[k]];
        p.schedule = code;
        p.stream = s;
        Z[k].reset(new SolveSetup());
        hms_status rc = setup_solve(cnfs[idx[k]], &p, *Z[k]);
        if (rc) return rc;
    }
    const hms_solve_params& p0 = params[idx[0]];
    const int32_t T = p0.steps, K = p0.eval_every, R = p0.restarts;
    const int sched = Z[0]->sh.sched;
    const int opt = Z[0]->L.opt;
    for (int32_t k = 1; k < cnt; ++k)
        if (Z[k]->sh.sched != sched || Z[k]->sh.U != Z[0]->sh.U || Z[k]->sh.Ub != Z[0]->sh.Ub || Z[k]->L.opt != opt ||
            Z[k]->sh.B.R != R)
            return fail(HMS_ERR_ARG, "the instances of a grouped launch must share one schedule");
    // argument arrays and running block counts
    std::vector<hms::FwdArgs> fa(cnt);
    std::vector<hms::BwdArgs> ba0(cnt), ba1(cnt);
    std::vector<hms::ReduceArgs> ra(cnt);
    std::vector<int32_t> b0[5];
    for (auto& v : b0) v.assign(1, 0);
    const int32_t gx = (R + 63) / 64;
    for (int32_t k = 0; k < cnt; ++k) {
        const Shape& sh = Z[k]->sh;
        const hms::HostPlan& P = cnfs[idx[k]]->plan;
        fa[k] = Z[k]->L.fa;
        ba0[k] = ba1[k] = Z[k]->L.ba;
        ba0[k].eval = 0;
        ba1[k].eval = 1;
        ra[k] = Z[k]->L.ra;
        const int64_t nblk[5] = {
            std::max<int64_t>(sh.fwd_blocks, 1),  // block 0 publishes the step scalars
            std::max<int64_t>(sh.bwd_blocks, 1),  // block 0 advances the step counter
            (int64_t)P.n_heavy_wide * R + ((int64_t)(P.n_heavy - P.n_heavy_wide) * R + 15) / 16,
            ra[k].n_chunks > 0 ? (int64_t)gx * ra[k].n_chunks : 0, (int64_t)gx};
        for (int j = 0; j < 5; ++j) {
            const int64_t tot = (int64_t)b0[j].back() + nblk[j];
            if (tot >= INT32_MAX / 2) return fail(HMS_ERR_TOO_LARGE, "too many work units in one batched launch");
            b0[j].push_back((int32_t)tot);
        }
    }
    Layout lay;
    const size_t o_fa = lay.add(sizeof(hms::FwdArgs) * cnt);
    const size_t o_b0 = lay.add(sizeof(hms::BwdArgs) * cnt);
    const size_t o_b1 = lay.add(sizeof(hms::BwdArgs) * cnt);
    const size_t o_ra = lay.add(sizeof(hms::ReduceArgs) * cnt);
    size_t o_blk[5];
    for (int j = 0; j < 5; ++j) o_blk[j] = lay.add(sizeof(int32_t) * (cnt + 1));
    Arena A;
    A.s = s;
    HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
    SyncOnExit args_done{s};
    HIPTRY(hipMemcpyAsync(A.base + o_fa, fa.data(), sizeof(hms::FwdArgs) * cnt, hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(A.base + o_b0, ba0.data(), sizeof(hms::BwdArgs) * cnt, hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(A.base + o_b1, ba1.data(), sizeof(hms::BwdArgs) * cnt, hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(A.base + o_ra, ra.data(), sizeof(hms::ReduceArgs) * cnt, hipMemcpyHostToDevice, s));
    for (int j = 0; j < 5; ++j)
        HIPTRY(hipMemcpyAsync(A.base + o_blk[j], b0[j].data(), sizeof(int32_t) * (cnt + 1), hipMemcpyHostToDevice, s));
    HIPTRY(hipStreamSynchronize(s));  // the host vectors above are temporaries
    auto ml = [&](size_t o_args, int j) {
        return hms::MultiLaunch{A.at<void>(o_args), A.at<int32_t>(o_blk[j]), cnt, b0[j].back()};
    };
    const hms::MultiLaunch mf = ml(o_fa, 0), mb0 = ml(o_b0, 1), mb1 = ml(o_b1, 1), mc0 = ml(o_b0, 2),
                           mc1 = ml(o_b1, 2), mr1 = ml(o_ra, 3), mr2 = ml(o_ra, 4);
    auto step = [&](bool eval, hipStream_t st) -> hipError_t {
        hipError_t e = hms::launch_fwd_multi(sched, eval, mf, st);
        if (e == hipSuccess && eval) e = hms::launch_reduce_multi(mr1, mr2, st);
        if (e == hipSuccess) e = hms::launch_bwd_multi(sched, opt, eval ? mb1 : mb0, st);
        if (e == hipSuccess) e = hms::launch_combine_multi(opt, eval ? mc1 : mc0, st);
        return e;
    };

    Events E;
    for (int i = 0; i < 2; ++i) HIPTRY(hipEventCreate(&E.e[i]));
    HIPTRY(hipEventRecord(E.e[0], s));
    int32_t done = 0;
    const int32_t B = graph_body(K);
    if (p0.use_graph && T >= 2 * B) {
        hipStream_t cs = nullptr;
        HIPTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        struct GFree {
            hipStream_t user;
            hipStream_t& s;
            hipGraph_t& g;
            hipGraphExec_t& x;
            ~GFree() {
                (void)hipStreamSynchronize(user);
                if (x) (void)hipGraphExecDestroy(x);
                if (g) (void)hipGraphDestroy(g);
                if (s) (void)hipStreamDestroy(s);
            }
        } gf{s, cs, graph, exec};
        HIPTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        hipError_t ce = hipSuccess;
        for (int32_t i = 0; i < B && ce == hipSuccess; ++i) ce = step(i % K == 0, cs);
        hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (ce != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(ce));
        if (ee != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(ee));
        HIPTRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        for (int32_t r = 0; r < T / B; ++r) {
            HIPTRY(hipGraphLaunch(exec, s));
            done += B;
        }
    }
    for (; done < T; ++done) HIPTRY(step(done % K == 0, s));
    for (int32_t k = 0; k < cnt; ++k) HIPTRY(count_final(cnfs[idx[k]], *Z[k], s));
    HIPTRY(hipEventRecord(E.e[1], s));
    HIPTRY(hipStreamSynchronize(s));
    float ms = 0.0f;
    HIPTRY(hipEventElapsedTime(&ms, E.e[0], E.e[1]));
    hms_status worst = HMS_OK;
    std::string msg;
    for (int32_t k = 0; k < cnt; ++k) {
        hms_status st = read_result(cnfs[idx[k]], *Z[k], done, ms, s, &results[idx[k]]);
        if (statuses) statuses[idx[k]] = st;
        if (st && !worst) {
            worst = st;
            msg = "instance " + std::to_string(idx[k]) + ": " + g_err;
        }
    }
    if (worst) return fail(worst, msg);
    return HMS_OK;
}

}  // namespace

extern "C" {

hms_status hms_solve(const hms_cnf* cnf, const hms_solve_params* p, hms_solve_result* res) {
    g_err.clear();
    if (check_cnf(cnf) || !p || !res) return fail(HMS_ERR_ARG, "null argument");
    if (hms_status rc = check_resume(cnf, p, res)) return rc;
    DeviceGuard dg(cnf->device);
    hms_solve_params pr = *p;
    hms_status rc0 = resolve_schedule(cnf, p, pr.schedule);
    if (rc0) return rc0;
    p = &pr;
    if (p->schedule == kResidentId) {
        if (!resident_ok(cnf, p)) return fail(HMS_ERR_ARG, "the resident schedule does not fit this instance");
        if (p->restarts < 1 || p->steps < 0 || p->eval_every < 1)
            return fail(HMS_ERR_ARG, "restarts >= 1, steps >= 0 and eval_every >= 1 required");
        return solve_resident(cnf, p, res);
    }
    SolveSetup Z;
    rc0 = setup_solve(cnf, p, Z);
    if (rc0) return rc0;
    const int32_t T = p->steps, K = p->eval_every;
    hipStream_t s = (hipStream_t)p->stream;
    Arena ring;  // trajectory ring, written by the count reduction
    if (res->trace) {
        ring.s = s;
        HIPTRY(hipMallocAsync((void**)&ring.base, (size_t)res->trace_cap * p->restarts * sizeof(hms::TracePoint), s));
        Z.L.ra.trace = ring.at<hms::TracePoint>(0);
        Z.L.ra.trace_cap = res->trace_cap;
        Z.L.ra.trace_k = K;
        Z.L.ra.trace_base = (int32_t)(((int64_t)Z.step0 + K - 1) / K);
    }
    const Launch& L = Z.L;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    HIPTRY(hipEventCreate(&ev0));
    HIPTRY(hipEventCreate(&ev1));
    struct EvFree {
        hipEvent_t a, b;
        ~EvFree() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } evf{ev0, ev1};
    HIPTRY(hipEventRecord(ev0, s));

    const auto t_host0 = std::chrono::steady_clock::now();
    bool cancelled = false;
    auto over_time = [&]() {
        if (p->cancel && *p->cancel) {
            cancelled = true;
            return true;
        }
        if (p->time_limit_s <= 0) return false;
        double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_host0).count();
        return el >= p->time_limit_s;
    };
    const bool watch = p->time_limit_s > 0 || p->cancel != nullptr;  // poll at K-step boundaries

    // iteration numbers go on from a resumed state: t = s0 + done
    const int32_t s0 = Z.step0;
    int32_t done = 0;
    bool stopped = false;  // the time limit ran out or the caller cancelled
    // direct launches until `upto` steps are done; the watch is polled when
    // t reaches a multiple of K
    auto direct = [&](int32_t upto) -> hms_status {
        while (done < upto && !stopped) {
            HIPTRY(enqueue_step(L, (s0 + done) % K == 0, s));
            ++done;
            if (watch && (s0 + done) % K == 0) {
                HIPTRY(hipStreamSynchronize(s));
                stopped = over_time();
            }
        }
        return HMS_OK;
    };
    // up to the first multiple of K, so the graph body starts on one
    if (hms_status rc = direct(std::min(T, (K - s0 % K) % K))) return rc;
    // body of B steps (a multiple of K, starting at a multiple of K)
    const int32_t B = graph_body(K);
    if (p->use_graph && T - done >= 2 * B && !stopped) {
        hipStream_t cs = nullptr;
        HIPTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        struct GFree {
            hipStream_t user;
            hipStream_t& s;
            hipGraph_t& g;
            hipGraphExec_t& x;
            ~GFree() {
                (void)hipStreamSynchronize(user);  // replays may still be running
                if (x) (void)hipGraphExecDestroy(x);
                if (g) (void)hipGraphDestroy(g);
                if (s) (void)hipStreamDestroy(s);
            }
        } gf{s, cs, graph, exec};
        HIPTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        hipError_t ce = hipSuccess;
        for (int32_t i = 0; i < B && ce == hipSuccess; ++i) ce = enqueue_step(L, i % K == 0, cs);
        hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (ce != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(ce));
        if (ee != hipSuccess) return fail(HMS_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(ee));
        HIPTRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        const int32_t reps = (T - done) / B;
        for (int32_t r = 0; r < reps; ++r) {
            HIPTRY(hipGraphLaunch(exec, s));
            done += B;
            if (watch) {
                HIPTRY(hipStreamSynchronize(s));
                if ((stopped = over_time())) break;
            }
        }
    }
    if (hms_status rc = direct(T)) return rc;
    // x_T is always counted
    HIPTRY(count_final(cnf, Z, s));
    HIPTRY(hipEventRecord(ev1, s));
    HIPTRY(hipStreamSynchronize(s));
    float ms = 0.0f;
    HIPTRY(hipEventElapsedTime(&ms, ev0, ev1));
    const hms_status rr = read_result(cnf, Z, done, ms, s, res);
    if (res->trace) {
        const hms_status rt = read_trace(Z.L.ra.trace, p->restarts, K, Z.step0, Z.step0 + done, s, res);
        if (rt) return rt;
    }
    if (cancelled && rr == HMS_OK) return fail(HMS_ERR_CANCELLED, "cancelled by the caller; the best so far is filled");
    return rr;
}

hms_status hms_time_kernels(const hms_cnf* cnf, const hms_solve_params* p, int32_t iters, double* fwd_ms,
                            double* bwd_ms, double* step_ms) {
    g_err.clear();
    if (check_cnf(cnf) || !p || iters < 1) return fail(HMS_ERR_ARG, "null argument or iters < 1");
    DeviceGuard dg(cnf->device);
    hms_solve_params pr = *p;
    pr.resume = nullptr;  // timing starts from the seed or x0
    hms_status rc0 = resolve_schedule(cnf, p, pr.schedule);
    if (rc0) return rc0;
    p = &pr;
    if (p->schedule == kResidentId) {
        if (!resident_ok(cnf, p)) return fail(HMS_ERR_ARG, "the resident schedule does not fit this instance");
        double ms = 0;
        hms_status rc = time_resident(cnf, p, iters, ms);
        if (rc) return rc;
        if (fwd_ms) *fwd_ms = 0.0;
        if (bwd_ms) *bwd_ms = 0.0;
        if (step_ms) *step_ms = ms;
        return HMS_OK;
    }
    SolveSetup Z;
    rc0 = setup_solve(cnf, p, Z);
    if (rc0) return rc0;
    hipStream_t s = (hipStream_t)p->stream;
    const Launch& L = Z.L;
    Events E;
    for (auto& e : E.e) HIPTRY(hipEventCreate(&e));
    // one warm step so every code object is resident
    HIPTRY(enqueue_step(L, false, s));
    HIPTRY(hipEventRecord(E.e[0], s));
    for (int32_t i = 0; i < iters; ++i) HIPTRY(hms::launch_fwd(Z.sh.sched, false, L.fa, Z.sh.fwd_blocks, s));
    HIPTRY(hipEventRecord(E.e[1], s));
    for (int32_t i = 0; i < iters; ++i) {
        HIPTRY(hms::launch_bwd(Z.sh.sched, L.opt, L.ba, Z.sh.bwd_blocks, s));
        HIPTRY(hms::launch_combine(L.opt, L.ba, s));
    }
    HIPTRY(hipEventRecord(E.e[2], s));
    for (int32_t i = 0; i < iters; ++i) HIPTRY(enqueue_step(L, false, s));
    HIPTRY(hipEventRecord(E.e[3], s));
    HIPTRY(hipStreamSynchronize(s));
    float a = 0, b = 0, c = 0;
    HIPTRY(hipEventElapsedTime(&a, E.e[0], E.e[1]));
    HIPTRY(hipEventElapsedTime(&b, E.e[1], E.e[2]));
    HIPTRY(hipEventElapsedTime(&c, E.e[2], E.e[3]));
    if (fwd_ms) *fwd_ms = a / iters;
    if (bwd_ms) *bwd_ms = b / iters;
    if (step_ms) *step_ms = c / iters;
    return HMS_OK;
}

// Batched solve: every instance that fits the resident solver runs in shared
// launches (one workgroup per (instance, restart), grouped by LDS size so
// each launch wastes at most half its LDS), the others one after the other on
// the tiled path.  Each result is bitwise what hms_solve gives alone.
hms_status hms_solve_batch(const hms_cnf* const* cnfs, const hms_solve_params* params, int32_t count,
                           hms_solve_result* results, hms_status* statuses) {
    g_err.clear();
    if (count < 0 || (count > 0 && (!cnfs || !params || !results))) return fail(HMS_ERR_ARG, "null argument");
    if (count == 0) return HMS_OK;
    if (statuses)
        for (int32_t i = 0; i < count; ++i) statuses[i] = HMS_OK;
    hipStream_t s = (hipStream_t)params[0].stream;
    int dev = cnfs[0] ? cnfs[0]->device : -1;
    for (int32_t i = 0; i < count; ++i) {
        if (!cnfs[i]) return fail(HMS_ERR_ARG, "null instance handle");
        if (cnfs[i]->device != dev) return fail(HMS_ERR_ARG, "all instances of a batch must be on one device");
        const hms_solve_params& p = params[i];
        if (p.restarts < 1 || p.steps < 0 || p.eval_every < 1 || (p.optimizer != HMS_ADAM && p.optimizer != HMS_SGD) ||
            (p.loss_mode != HMS_LOSS_UNSAT && p.loss_mode != HMS_LOSS_ALL))
            return fail(HMS_ERR_ARG, "invalid parameters for instance " + std::to_string(i));
    }
    DeviceGuard dg(dev);
    std::vector<int32_t> res_idx, tiled_idx, alone;
    for (int32_t i = 0; i < count; ++i) {
        // a resumed solve, or one that hands back its state or its trajectory, runs as hms_solve
        if (params[i].resume != nullptr || results[i].state != nullptr || results[i].trace != nullptr) {
            alone.push_back(i);
            continue;
        }
        const bool want_res = params[i].schedule == kResidentId ||
                              (params[i].schedule == 0 && resident_preferred(cnfs[i], &params[i]));
        if (want_res && resident_ok(cnfs[i], &params[i])) res_idx.push_back(i);
        else tiled_idx.push_back(i);
    }
    hms_status worst = HMS_OK;
    std::string worst_msg;
    if (!res_idx.empty()) {
        std::sort(res_idx.begin(), res_idx.end(), [&](int32_t a, int32_t b) {
            return resident_lds(cnfs[a]) > resident_lds(cnfs[b]);
        });
        // device arena: descriptors, then each instance's outputs
        Layout lay;
        const size_t o_desc = lay.add(sizeof(hms::SmallDesc) * res_idx.size());
        std::vector<SmallOut> outs(res_idx.size());
        for (size_t k = 0; k < res_idx.size(); ++k)
            outs[k] = layout_small_out(cnfs[res_idx[k]]->plan, params[res_idx[k]].restarts, lay);
        // host destinations of the read-back copies, declared before the
        // guard that waits for the stream (an early return cannot free them
        // under a copy)
        std::vector<std::vector<int64_t>> best(res_idx.size());
        std::vector<std::vector<int32_t>> step(res_idx.size());
        std::vector<std::vector<double>> loss(res_idx.size());
        Arena A;
        A.s = s;
        HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
        std::vector<hms::SmallDesc> D(res_idx.size());
        for (size_t k = 0; k < res_idx.size(); ++k) {
            const int32_t i = res_idx[k];
            D[k] = make_desc(cnfs[i], &params[i]);
            D[k].best_a = A.at<uint8_t>(outs[k].o_best_a);
            D[k].best = A.at<int64_t>(outs[k].o_best);
            D[k].best_step = A.at<int32_t>(outs[k].o_step);
            D[k].final_loss = A.at<double>(outs[k].o_loss);
            D[k].x_final = results[i].x_final;
        }
        // launches: consecutive instances whose LDS need is within 2x of the first
        size_t k0 = 0;
        std::vector<std::pair<size_t, size_t>> groups;
        while (k0 < res_idx.size()) {
            const size_t big = resident_lds(cnfs[res_idx[k0]]);
            size_t k1 = k0 + 1;
            while (k1 < res_idx.size() && 2 * resident_lds(cnfs[res_idx[k1]]) >= big) ++k1;
            groups.emplace_back(k0, k1);
            k0 = k1;
        }
        for (auto& g : groups) {
            int32_t blocks = 0;
            for (size_t k = g.first; k < g.second; ++k) {
                D[k].block0 = blocks;
                blocks += params[res_idx[k]].restarts;
            }
        }
        SyncOnExit d_done{s};
        HIPTRY(hipMemcpyAsync(A.base + o_desc, D.data(), sizeof(hms::SmallDesc) * D.size(), hipMemcpyHostToDevice, s));
        Events E;
        for (int i = 0; i < 2; ++i) HIPTRY(hipEventCreate(&E.e[i]));
        HIPTRY(hipEventRecord(E.e[0], s));
        for (auto& g : groups) {
            int32_t blocks = 0;
            int32_t stage = 3;  // the sides every instance of the group stages
            int32_t rows = 0;
            for (size_t k = g.first; k < g.second; ++k) {
                blocks += params[res_idx[k]].restarts;
                stage &= D[k].stage;
                rows = std::max(rows, resident_rows(cnfs[res_idx[k]]));
            }
            bool reg = true;  // every instance keeps its rows in registers
            for (size_t k = g.first; k < g.second; ++k) reg = reg && hms::small_reg_ok(cnfs[res_idx[k]]->plan, rows);
            HIPTRY(hms::launch_small(A.at<hms::SmallDesc>(o_desc) + g.first, (int32_t)(g.second - g.first), blocks,
                                     resident_lds(cnfs[res_idx[g.first]]), lds_limit(dev), stage, rows, reg, s));
        }
        HIPTRY(hipEventRecord(E.e[1], s));
        // read back every resident result
        for (size_t k = 0; k < res_idx.size(); ++k) {
            const int32_t R = params[res_idx[k]].restarts;
            best[k].resize(R);
            step[k].resize(R);
            loss[k].resize(R);
            HIPTRY(hipMemcpyAsync(best[k].data(), D[k].best, R * 8, hipMemcpyDeviceToHost, s));
            HIPTRY(hipMemcpyAsync(step[k].data(), D[k].best_step, R * 4, hipMemcpyDeviceToHost, s));
            HIPTRY(hipMemcpyAsync(loss[k].data(), D[k].final_loss, R * 8, hipMemcpyDeviceToHost, s));
        }
        HIPTRY(hipStreamSynchronize(s));
        float ms = 0;
        HIPTRY(hipEventElapsedTime(&ms, E.e[0], E.e[1]));
        for (size_t k = 0; k < res_idx.size(); ++k) {
            const int32_t i = res_idx[k];
            const int32_t R = params[i].restarts;
            const hms::HostPlan& P = cnfs[i]->plan;
            hms_solve_result& res = results[i];
            int32_t br = 0;
            for (int32_t r = 1; r < R; ++r)
                if (best[k][r] < best[k][br]) br = r;
            if (res.best_assignment && P.n > 0)
                HIPTRY(hipMemcpyAsync(res.best_assignment, D[k].best_a + (size_t)br * P.n, P.n, hipMemcpyDeviceToHost,
                                      s));
            res.best_cost = best[k][br];
            res.best_restart = br;
            res.best_step = step[k][br];
            res.steps_done = params[i].steps;
            res.schedule = kResidentId;
            res.final_loss = loss[k][br];
            res.device_ms = ms;
            if (res.restart_best) std::memcpy(res.restart_best, best[k].data(), R * 8);
            if (res.restart_step) std::memcpy(res.restart_step, step[k].data(), R * 4);
            if (res.restart_loss) std::memcpy(res.restart_loss, loss[k].data(), R * 8);
            hms_status st = HMS_OK;
            for (int32_t r = 0; r < R; ++r)
                if (!std::isfinite(loss[k][r])) st = HMS_ERR_NONFINITE;
            if (statuses) statuses[i] = st;
            if (st && !worst) {
                worst = st;
                worst_msg = "instance " + std::to_string(i) + ": the loss at the final iterate is not finite";
            }
        }
        HIPTRY(hipStreamSynchronize(s));
    }
    // tiled instances: groups that share restarts, steps, counting period,
    // optimizer, loss mode and requested schedule run together (largest
    // first, at most kGroup per launch) with the schedule of their largest
    // instance; a group of one, or a solve with a time limit, runs alone
    constexpr size_t kGroup = 64;
    std::map<std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>, std::vector<int32_t>> groups;
    for (int32_t i : tiled_idx) {
        const hms_solve_params& p = params[i];
        if (p.time_limit_s > 0 || p.cancel != nullptr) {
            alone.push_back(i);
            continue;
        }
        const int32_t sch = p.schedule == kResidentId ? 0 : p.schedule;
        groups[std::make_tuple(p.restarts, p.steps, p.eval_every, p.optimizer, p.loss_mode, sch)].push_back(i);
    }
    auto note = [&](hms_status st, int32_t i) {
        if (st && !worst) {
            worst = st;
            worst_msg = "instance " + std::to_string(i) + ": " + g_err;
        }
    };
    for (auto& kv : groups) {
        std::vector<int32_t>& g = kv.second;
        std::stable_sort(g.begin(), g.end(), [&](int32_t a, int32_t b) { return cnfs[a]->plan.nnz > cnfs[b]->plan.nnz; });
        for (size_t k0 = 0; k0 < g.size(); k0 += kGroup) {
            const int32_t cnt = (int32_t)std::min(kGroup, g.size() - k0);
            if (cnt == 1) {
                alone.push_back(g[k0]);
                continue;
            }
            hms_solve_params p = params[g[k0]];
            p.stream = params[0].stream;
            if (p.schedule == kResidentId) p.schedule = 0;
            int32_t code = 0;
            hms_status st = resolve_schedule(cnfs[g[k0]], &p, code);
            if (!st && code == kResidentId) code = 0;
            // one explicit schedule for the whole group (the automatic choice
            // depends on the instance)
            Shape sh0;
            if (!st) st = make_shape(cnfs[g[k0]]->plan, p.restarts, code, p.loss_mode, sh0);
            if (!st && p.schedule == 0 && sh0.slot) {
                // the slot schedules carry two more entry-sized streams; once a
                // group's instances together pass 2^24 nonzeros (their streams
                // no longer stay in the Infinity Cache) the bitset schedule
                // runs the group faster (16 instances of 60000-200000
                // variables: 86.6 against 78.8 instances/s)
                int64_t nnz = 0;
                for (int32_t k = 0; k < cnt; ++k) nnz += cnfs[g[k0 + k]]->plan.nnz;
                if (nnz > (int64_t(1) << 24)) st = make_shape(cnfs[g[k0]]->plan, p.restarts, 37 | (64 << 8), p.loss_mode, sh0);
            }
            if (!st) st = solve_tiled_group(cnfs, params, g.data() + k0, cnt, sh0.code, s, results, statuses);
            if (st) {
                if (statuses)
                    for (int32_t k = 0; k < cnt; ++k)
                        if (statuses[g[k0 + k]] == HMS_OK) statuses[g[k0 + k]] = st;
                note(st, g[k0]);
            }
        }
    }
    for (int32_t i : alone) {
        hms_solve_params p = params[i];
        p.stream = params[0].stream;
        if (p.schedule == kResidentId) p.schedule = 0;
        hms_status st = hms_solve(cnfs[i], &p, &results[i]);
        if (statuses) statuses[i] = st;
        note(st, i);
    }
    if (worst) return fail(worst, worst_msg);
    g_err.clear();
    return HMS_OK;
}

hms_status hms_tune_candidates(int32_t restarts, int32_t loss_mode, int32_t* codes, int32_t cap, int32_t* count) {
    g_err.clear();
    if (!count || cap < 0 || (cap > 0 && !codes)) return fail(HMS_ERR_ARG, "null argument or negative capacity");
    if (restarts < 1) return fail(HMS_ERR_ARG, "restarts >= 1 required");
    if (loss_mode != HMS_LOSS_UNSAT && loss_mode != HMS_LOSS_ALL) return fail(HMS_ERR_ARG, "unknown loss mode");
    const std::vector<int32_t> c = tune_candidates(restarts, loss_mode);
    *count = (int32_t)c.size();
    for (size_t i = 0; i < c.size() && (int32_t)i < cap; ++i) codes[i] = c[i];
    return HMS_OK;
}

int32_t hms_schedule_count(void) { return hms::kNumSchedules; }

hms_status hms_tune(const hms_cnf* cnf, const hms_solve_params* params, int32_t iters, int32_t* schedule,
                    double* step_ms) {
    g_err.clear();
    if (check_cnf(cnf) || !params || iters < 1) return fail(HMS_ERR_ARG, "null argument or iters < 1");
    DeviceGuard dg(cnf->device);
    int32_t best = 0;
    double ms = 0;
    hms_status rc = tune(cnf, params, iters, best, ms);
    if (rc) return rc;
    if (schedule) *schedule = best;
    if (step_ms) *step_ms = ms;
    return HMS_OK;
}

}  // extern "C"

namespace {

// Workspace of hms_eval_relaxed_noalloc: a fixed device array, one copy per
// GPU (each GPU holds it until the process ends).  Host code must never use
// the array's name as an address: its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};  // device address of `scratch` on each GPU, once known

// Device address of the workspace on `dev` (the current device).
hms_status scratch_on(int dev, char*& ptr) {
    if (dev < 0 || dev >= 64) return fail(HMS_ERR_DEVICE, "device index out of range for the fixed workspace");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(HMS_ERR_DEVICE, std::string("hipGetSymbolAddress of the fixed workspace: ") +
                                            hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    ptr = static_cast<char*>(g_scratch_ptr[dev]);
    return HMS_OK;
}

// One evaluation of the relaxed objective (hms_eval_relaxed).  With `fixed`
// the workspace is that device memory (cap bytes) and loss / unsat are
// DEVICE outputs, so nothing is allocated and nothing waits; otherwise the
// workspace is a stream-ordered allocation of this call and loss / unsat are
// HOST outputs.
hms_status eval_relaxed_impl(const hms_cnf* cnf, const float* x, int32_t R, int32_t loss_mode, double* loss,
                             float* grad, int64_t* unsat, void* stream, char* fixed, size_t cap) {
    if (check_cnf(cnf) || (!x && cnf->plan.n > 0)) return fail(HMS_ERR_ARG, "null argument");
    if (R < 1) return fail(HMS_ERR_ARG, "restarts >= 1 required");
    if (loss_mode != HMS_LOSS_UNSAT && loss_mode != HMS_LOSS_ALL) return fail(HMS_ERR_ARG, "unknown loss mode");
    const hms::HostPlan& P = cnf->plan;
    hipStream_t s = (hipStream_t)stream;
    Shape sh;
    // one evaluation gains nothing from the occurrence slots (its forward
    // pays for them) and they would take workspace
    hms_status rc = make_shape(P, R, 0, loss_mode, sh, true, false);
    if (rc) return rc;
    const bool want_g = grad != nullptr;
    Layout lay;
    size_t off[kOffN];
    layout_state(P, sh, false, want_g, false, lay, off);
    Arena A;
    A.s = s;
    if (fixed) {
        if (lay.off > cap)
            return fail(HMS_ERR_TOO_LARGE, "this evaluation needs " + std::to_string(lay.off) +
                                               " bytes of workspace, more than the " + std::to_string(cap) +
                                               " of the allocation-free variant");
        A.base = fixed;
        A.owns = false;
    } else {
        HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
    }
    // host outputs are written by queued copies: an early return waits (the
    // allocation-free variant has device outputs only and never waits)
    SyncOnExit outs_done{s, fixed == nullptr};
    // every piece the kernels read is written first (init kernel, forward
    // pass), so a reused workspace needs no clearing
    State S = bind_state(A, off, false, want_g, false);
    hms::InitArgs ia = make_init(cnf, sh, S);
    ia.x0 = x;
    HIPTRY(hms::launch_init(ia, s));
    Launch L = make_launch(cnf, sh, S, hms::kGrad, loss_mode, 0.f, 0.9f, 0.999f, 1e-8f);
    L.ra.track = 0;
    HIPTRY(hms::launch_fwd(sh.sched, true, L.fa, sh.fwd_blocks, s));
    HIPTRY(hms::launch_reduce(L.ra, s));
    if (want_g) {
        HIPTRY(hms::launch_bwd(sh.sched, hms::kGrad, L.ba, sh.bwd_blocks, s));
        HIPTRY(hms::launch_combine(hms::kGrad, L.ba, s));
        HIPTRY(hms::launch_scatter(P.n, P.n_act, sh.B, cnf->var_old, S.g, grad, s));
    }
    const hipMemcpyKind kind = fixed ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (loss) HIPTRY(hipMemcpyAsync(loss, S.cur_loss, (size_t)R * 8, kind, s));
    if (unsat) HIPTRY(hipMemcpyAsync(unsat, S.cur_count, (size_t)R * 8, kind, s));
    if (!fixed && (loss || unsat)) HIPTRY(hipStreamSynchronize(s));
    return HMS_OK;
}

}  // namespace

extern "C" {

hms_status hms_eval_relaxed(const hms_cnf* cnf, const float* x, int32_t R, int32_t loss_mode, double* loss,
                            float* grad, int64_t* unsat, void* stream) {
    g_err.clear();
    if (check_cnf(cnf)) return fail(HMS_ERR_ARG, "null instance handle");
    DeviceGuard dg(cnf->device);
    return eval_relaxed_impl(cnf, x, R, loss_mode, loss, grad, unsat, stream, nullptr, 0);
}

hms_status hms_eval_relaxed_noalloc(const hms_cnf* cnf, const float* x, int32_t R, int32_t loss_mode, double* loss,
                                    float* grad, int64_t* unsat, void* stream) {
    g_err.clear();
    if (check_cnf(cnf)) return fail(HMS_ERR_ARG, "null instance handle");
    DeviceGuard dg(cnf->device);
    char* ws = nullptr;
    hms_status rc = scratch_on(cnf->device, ws);
    if (rc) return rc;
    return eval_relaxed_impl(cnf, x, R, loss_mode, loss, grad, unsat, stream, ws, kScratchBytes);
}

// ---- differentiable forward / backward ---------------------------------------
// Both use the automatic schedule for R without the bitset, so the adjoint a
// forward saves is the array the backward reads.
hms_status adjoint_shape(const hms_cnf* cnf, int32_t R, int32_t loss_mode, Shape& sh) {
    if (R < 1) return fail(HMS_ERR_ARG, "restarts >= 1 required");
    if (loss_mode != HMS_LOSS_UNSAT && loss_mode != HMS_LOSS_ALL) return fail(HMS_ERR_ARG, "unknown loss mode");
    return make_shape(cnf->plan, R, 0, loss_mode, sh, false);
}

hms_status hms_adjoint_bytes(const hms_cnf* cnf, int32_t R, int64_t* bytes) {
    g_err.clear();
    if (check_cnf(cnf) || !bytes) return fail(HMS_ERR_ARG, "null argument");
    Shape sh;
    hms_status rc = adjoint_shape(cnf, R, HMS_LOSS_UNSAT, sh);
    if (rc) return rc;
    *bytes = (int64_t)sh.B.rows_a * sh.B.RG * sh.B.G * 4;
    return HMS_OK;
}

hms_status hms_forward(const hms_cnf* cnf, const float* x, int32_t R, int32_t loss_mode, double* loss,
                       int64_t* unsat, void* adjoint, void* stream) {
    g_err.clear();
    if (check_cnf(cnf) || (!x && cnf->plan.n > 0) || !loss) return fail(HMS_ERR_ARG, "null argument");
    const hms::HostPlan& P = cnf->plan;
    DeviceGuard dg(cnf->device);
    hipStream_t s = (hipStream_t)stream;
    Shape sh;
    hms_status rc = adjoint_shape(cnf, R, loss_mode, sh);
    if (rc) return rc;
    Layout lay;
    size_t off[kOffN];
    layout_state(P, sh, false, false, false, lay, off);
    Arena A;
    A.s = s;
    HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
    State S = bind_state(A, off, false, false, false);
    if (adjoint) S.a = static_cast<float*>(adjoint);
    hms::InitArgs ia = make_init(cnf, sh, S);
    ia.x0 = x;
    HIPTRY(hms::launch_init(ia, s));
    Launch L = make_launch(cnf, sh, S, hms::kGrad, loss_mode, 0.f, 0.9f, 0.999f, 1e-8f);
    L.ra.track = 0;
    HIPTRY(hms::launch_fwd(sh.sched, true, L.fa, sh.fwd_blocks, s));
    HIPTRY(hms::launch_reduce(L.ra, s));
    HIPTRY(hipMemcpyAsync(loss, S.cur_loss, (size_t)R * 8, hipMemcpyDeviceToDevice, s));
    if (unsat) HIPTRY(hipMemcpyAsync(unsat, S.cur_count, (size_t)R * 8, hipMemcpyDeviceToDevice, s));
    return HMS_OK;
}

hms_status hms_backward(const hms_cnf* cnf, const float* x, int32_t R, int32_t loss_mode, const void* adjoint,
                        const float* grad_loss, float* grad_x, void* stream) {
    g_err.clear();
    if (check_cnf(cnf) || (!x && cnf->plan.n > 0) || (!grad_x && cnf->plan.n > 0))
        return fail(HMS_ERR_ARG, "null argument");
    const hms::HostPlan& P = cnf->plan;
    DeviceGuard dg(cnf->device);
    hipStream_t s = (hipStream_t)stream;
    Shape sh;
    hms_status rc = adjoint_shape(cnf, R, loss_mode, sh);
    if (rc) return rc;
    Layout lay;
    size_t off[kOffN];
    layout_state(P, sh, false, true, false, lay, off);
    Arena A;
    A.s = s;
    HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
    State S = bind_state(A, off, false, true, false);
    if (adjoint) S.a = const_cast<float*>(static_cast<const float*>(adjoint));
    hms::InitArgs ia = make_init(cnf, sh, S);
    ia.x0 = x;
    if (adjoint) ia.a = nullptr;  // the saved adjoint is read-only here
    HIPTRY(hms::launch_init(ia, s));
    Launch L = make_launch(cnf, sh, S, hms::kGrad, loss_mode, 0.f, 0.9f, 0.999f, 1e-8f);
    if (!adjoint) HIPTRY(hms::launch_fwd(sh.sched, false, L.fa, sh.fwd_blocks, s));  // recompute the scores
    HIPTRY(hms::launch_bwd(sh.sched, hms::kGrad, L.ba, sh.bwd_blocks, s));
    HIPTRY(hms::launch_combine(hms::kGrad, L.ba, s));
    HIPTRY(hms::launch_scatter(P.n, P.n_act, sh.B, cnf->var_old, S.g, grad_x, s, grad_loss));
    return HMS_OK;
}

hms_status hms_evaluate(const hms_cnf* cnf, const uint8_t* assignment, int64_t* unsat, void* stream) {
    g_err.clear();
    if (check_cnf(cnf) || !unsat || (!assignment && cnf->plan.n > 0)) return fail(HMS_ERR_ARG, "null argument");
    const hms::HostPlan& P = cnf->plan;
    DeviceGuard dg(cnf->device);
    hipStream_t s = (hipStream_t)stream;
    Shape sh;
    hms_status rc = make_shape(P, 1, 1, HMS_LOSS_UNSAT, sh);
    if (rc) return rc;
    Layout lay;
    size_t off[kOffN];
    layout_state(P, sh, false, false, false, lay, off);
    const size_t o_in = lay.add((size_t)std::max(P.n, 1));
    Arena A;
    A.s = s;
    HIPTRY(hipMallocAsync((void**)&A.base, lay.off, s));
    State S = bind_state(A, off, false, false, false);
    uint8_t* d_in = A.at<uint8_t>(o_in);
    SyncOnExit in_done{s};  // the caller's buffers are in use until the stream drains
    if (P.n > 0) HIPTRY(hipMemcpyAsync(d_in, assignment, P.n, hipMemcpyHostToDevice, s));
    hms::InitArgs ia = make_init(cnf, sh, S);
    ia.assign0 = d_in;
    HIPTRY(hms::launch_init(ia, s));
    Launch L = make_launch(cnf, sh, S, hms::kGrad, HMS_LOSS_UNSAT, 0.f, 0.9f, 0.999f, 1e-8f);
    L.ra.track = 0;
    HIPTRY(hms::launch_fwd(sh.sched, true, L.fa, sh.fwd_blocks, s));
    HIPTRY(hms::launch_reduce(L.ra, s));
    HIPTRY(hipMemcpyAsync(unsat, S.cur_count, 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    return HMS_OK;
}

// ---- host-only plan view --------------------------------------------------
hms_status hms_plan_view_build(int32_t n_vars, const int32_t* lits, int64_t n_lits, hms_plan_view* out) {
    g_err.clear();
    if (!out) return fail(HMS_ERR_ARG, "null output");
    std::memset(out, 0, sizeof(*out));
    hms::HostPlan* P = new (std::nothrow) hms::HostPlan();
    if (!P) return fail(HMS_ERR_NOMEM, "host allocation failed");
    std::string err;
    int32_t rc = hms::build_plan(n_vars, lits, n_lits, nullptr, *P, err);
    if (rc) {
        delete P;
        return fail(rc, err);
    }
    hms::build_slots(*P);
    out->n = P->n;
    out->m = P->m;
    out->mk = P->mk;
    out->c_tiles = P->c_tiles;
    out->n_act = P->n_act;
    out->n_heavy = P->n_heavy;
    out->seg_rows = P->seg_rows;
    out->seg_tiles = P->seg_tiles;
    out->v_tiles = P->v_tiles;
    out->n_empty = P->m_empty;
    out->n_taut = P->m_taut;
    out->tile_rows = hms::kTile;
    out->seg_len = hms::kSeg;
    out->split_len = P->split_len;
    out->nnz = P->nnz;
    out->c_ent_len = (int64_t)P->c_ent.size();
    out->v_ent_len = (int64_t)P->v_ent.size();
    out->c_tile = reinterpret_cast<const uint32_t*>(P->c_tile.data());
    out->c_ent = P->c_ent.data();
    out->c_row_orig = P->c_row_orig.data();
    out->v_tile = reinterpret_cast<const uint32_t*>(P->v_tile.data());
    out->v_ent = P->v_ent.data();
    out->seg_first = P->seg_first.data();
    out->seg_row = P->seg_row.data();
    out->var_old = P->var_old.data();
    out->c_slot = P->c_slot.empty() ? nullptr : P->c_slot.data();
    out->priv = P;
    return HMS_OK;
}

void hms_plan_view_free(hms_plan_view* view) {
    if (!view) return;
    delete static_cast<hms::HostPlan*>(view->priv);
    std::memset(view, 0, sizeof(*view));
}

hms_status hms_cnf_slot_map(const hms_cnf* cnf, uint32_t* out, int64_t cap, int64_t* len) {
    g_err.clear();
    if (check_cnf(cnf) || !len) return fail(HMS_ERR_ARG, "null argument");
    *len = 0;
    if (!cnf->c_slot) return HMS_OK;
    const int64_t n = (int64_t)cnf->plan.c_ent.size();
    if (!out) {  // size query
        *len = n;
        return HMS_OK;
    }
    if (cap < n) return fail(HMS_ERR_ARG, "output array shorter than the clause side");
    DeviceGuard dg(cnf->device);
    HIPTRY(hipDeviceSynchronize());
    HIPTRY(hipMemcpy(out, cnf->c_slot, (size_t)n * 4, hipMemcpyDeviceToHost));
    *len = n;
    return HMS_OK;
}

}  // extern "C"
