// eqs_host.cpp -- context, workspace and solve drivers behind the eqsolve C ABI.
//
// A context owns, per equation set, the FP64 (and for the FP32 forms, FP32)
// Krylov vectors, tile partials and a device-resident SolveState, all sized
// once in eqsolve_create.  A solve call only updates the set's descriptor
// (the caller's pointers, tol, maxit) and enqueues kernels on the context's
// stream; the BiCGSTAB scalars never leave the device.  The host reads the
// small state block back once per chunk of iterations to decide what to
// enqueue next (more iterations, the true-residual recheck, the refinement
// update), and sizes the next chunk from the observed convergence rate, so
// a solve costs a handful of host round trips, not one per iteration.
//
// This mirrors the paper's runtime shape (arXiv 2211.15605, Sec. 2.2.1 and
// 2.2.2): state stays resident on the device between calls and only scalars
// cross the host boundary.

#include <hip/hip_runtime_api.h>

#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "eqs_internal.h"
#include "eqs_launch.h"
#include "eqs_static.h"
#include "eqsolve.h"

using namespace eqs;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 64 * 1024;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct SetHost {
    eqs_grid g;
    int n, plane;
    int S, KC, NKC, ntiles, nflat;
    int fS, fntiles, ford;  // the single-sync step's tiling (segments of fnt * cpt cells) and tile order
    // workspace offsets resolved to pointers
    double *r, *rh, *p[2], *v[2], *t, *y;
    double *as[6];
    double *s1, *t1, *f;
    double *dinv;
    float *as32[6];
    float *sym32[4];
    float *r32, *rh32, *p32[2], *v32[2], *t32, *d32;
    float *s1_32, *t1_32, *f32;
    double *partials;
    uint32_t *counter;
    // convergence-rate tracking for chunk sizing
    int last_iters;
    int kc_jacobi;   // planes per chunk of the Jacobi iteration (tuned); 0 until first re-tiling
    bool form_sym;   // the last solve ran the symmetric form of the single-sync step
    bool form_raw;   // the last solve ran the raw form of the single-sync step
    double last_log_rr;
};

int env_int(const char *name, int dflt) {
    const char *s = getenv(name);
    if (!s || !*s) return dflt;
    return atoi(s);
}

double env_double(const char *name, double dflt) {
    const char *s = getenv(name);
    if (!s || !*s) return dflt;
    return atof(s);
}

// Relative tolerance of each FP32 inner solve of the refinement.  FP32
// BiCGSTAB stops gaining true (FP64) residual reduction after about two to
// three decades on these systems, so solving each correction loosely and
// taking a few more outer steps minimises the total inner iterations.
double inner_tol() { return env_double("EQS_TOL_INNER", 3e-3); }

// Single-sync iteration: the relative gap between sigma taken directly and the
// expanded sigma a step ran with, above which the iteration starts afresh
// (FP64, FP32).
double sigma_tol(bool fp32) { return fp32 ? env_double("EQS_SIGMA_TOL32", 1e-2) : env_double("EQS_SIGMA_TOL", 1e-3); }

}  // namespace

struct eqs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int nsets = 0;
    int precision = 0;
    int cpt = 2;
    int max_nx = 1;
    // iteration scheme: one fused launch and one reduction per step (true), or
    // three launches and three reductions per step (false)
    bool sync1 = true;
    // exactly symmetric sets take the symmetric form of the single-sync step (EQS_SYM=0: never)
    int sym_on = 1;
    // threads per block of the single-sync step (256 or 512) and the dynamic LDS it may take
    int fnt = 256;
    size_t fused_lds_cap = kMaxLds;
    SetHost sets[kMaxSets] = {};
    SetDesc *h_desc = nullptr;
    SetDesc *d_desc = nullptr;
    SolveState *h_state = nullptr;
    SolveState *d_state = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool broken = false;
    uint64_t launches = 0, readbacks = 0;
    // optional per-launch event timing (diagnostics)
    uint32_t profile_mask = 0;  // bit k: time launches of kernel kind k
    int profile_every = 1;      // time every n-th launch of a timed kind
    int64_t kseen[2 * 32] = {0};  // launches of each kind since profiling started
    int kpos[2 * 32] = {0};       // launches of each kind since the last readback
    std::vector<int> ev_pos;      // position of each timed launch since the last readback
    // captured iteration chunks: (first set, set count, transpose, fp32, symmetric form) -> graphs
    // of 2^k iterations
    bool use_graphs = true;
    bool use_small = true;      // one-block persistent solve for tiny FP64 sets (EQS_SMALL=0 disables)
    hipStream_t capture_stream = nullptr;
    std::map<std::tuple<int, int, bool, bool, int>, std::array<hipGraphExec_t, 9>> graphs;
    // the single-sync step's products of the FP64 forward solves: 0 from the coefficients of
    // A D^-1 (a per-solve scale pass writes them), 1 from the caller's coefficients (no scale
    // pass; eqsolve_set_step_form)
    int step_form = 0;
    bool trace = false;         // print the state at every readback (EQS_TRACE=1)
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_kind;     // pending (start, stop) pairs: kind per pair
    size_t ev_used = 0;
    int64_t kcount[2 * 32] = {0};
    double kms[2 * 32] = {0};
    // multigrid preconditioner of the FP64 forward solves (eqsolve_set_preconditioner)
    int precond = 0;                        // EQS_PRECOND_*
    MgParams mgp{0.8, 1.0, 30, 512};
    std::vector<std::vector<MgLevel>> mg;   // per set: the level table (host copy)
    MgLevel *d_mg = nullptr;                // device: nsets x kMgMaxLevels
    void *mg_ws = nullptr;
    std::map<std::pair<int, int>, std::array<hipGraphExec_t, 4>> graphs_mg;  // per run: 2^k preconditioned iterations
};

namespace {

#define EQS_HIP(call)                                 \
    do {                                              \
        if ((call) != hipSuccess) {                   \
            (void)hipGetLastError();                  \
            c->broken = true;                         \
            return EQS_ERR_HIP;                       \
        }                                             \
    } while (0)

// widest row a stencil pass stages (one row on each side of a segment, in LDS)
constexpr int kMaxNx = 1024;

bool grid_ok(const eqs_grid &g) {
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > kMaxNx) return false;
    const long long n = (long long)g.nx * g.ny * g.nz;
    return n < (1ll << 31) - (1ll << 20);
}

// the single-sync step's tiles: segments of fnt * cpt cells, the march's chunks
void fused_tiling(SetHost &s, int cpt, int fnt, int ford) {
    const int Q = fnt * cpt;
    s.fS = (s.plane + Q - 1) / Q;
    s.fntiles = s.fS * s.NKC;
    s.ford = ford ? 1 : 0;
}

// tiles: segments of Q = 256*cpt cells per plane, KC planes per chunk
void choose_tiling(SetHost &s, int cpt, int fnt) {
    const int Q = kBlock * cpt;
    s.S = (s.plane + Q - 1) / Q;
    const int target = std::max(1, env_int("EQS_TILE_TARGET", 1024));
    int kc = env_int("EQS_KC", 0);
    if (kc <= 0) {
        const long long want = ((long long)s.S * s.g.nz + target - 1) / target;
        kc = (int)std::min<long long>(std::max<long long>(want, 1), 32);
    }
    s.KC = std::min(kc, s.g.nz);
    s.NKC = (s.g.nz + s.KC - 1) / s.KC;
    s.ntiles = s.S * s.NKC;
    const int fmax = std::min(std::max(1, env_int("EQS_FLAT_MAX", 1024)), kMaxFlatBlocks);
    s.nflat = std::min((s.n + kFlatChunk - 1) / kFlatChunk, fmax);
    fused_tiling(s, cpt, fnt, env_int("EQS_FORD", 0));
}

// explicit tiling (tuner, tuning cache)
void set_tiling(SetHost &s, int cpt, int kc, int nflat, int fnt, int ford) {
    const int Q = kBlock * cpt;
    s.S = (s.plane + Q - 1) / Q;
    s.KC = std::max(1, std::min(kc, s.g.nz));
    s.NKC = (s.g.nz + s.KC - 1) / s.KC;
    s.ntiles = s.S * s.NKC;
    s.nflat = std::max(1, std::min(nflat, std::min((s.n + kFlatChunk - 1) / kFlatChunk, kMaxFlatBlocks)));
    fused_tiling(s, cpt, fnt, ford);
}

// partial sums are sized for any tiling the tuner may choose
size_t max_partials(const SetHost &s) {
    const long long tiles = (long long)((s.plane + kBlock - 1) / kBlock) * s.g.nz;  // cpt = 1, KC = 1
    return (size_t)std::max<long long>(tiles, kMaxFlatBlocks);
}

// device workspace of one set: the FP64 vectors and scaled coefficients (18 arrays), for the
// FP32 forms their FP32 counterparts (21 arrays), `partial_rows` rows of reduction partials and
// the ticket counter
size_t set_ws_bytes(const SetHost &h, bool f32, size_t partial_rows) {
    size_t bytes = 18 * align_up((size_t)h.n * 8);   // r, r^, p[2], v[2], t, y, 6 scaled coefficients, s1, t1, f, 1/a_P
    if (f32) bytes += 21 * align_up((size_t)h.n * 4);  // the same in FP32 (d = the inner iterate), a_E, a_N, a_T
    bytes += align_up(partial_rows * kMaxRed * 8);
    bytes += kAlign;  // counter
    return bytes;
}

// lay the set's workspace out from q (set_ws_bytes(h, f32, partial_rows) bytes, 256-byte aligned)
void carve_set(SetHost &h, char *q, bool f32, size_t partial_rows) {
    auto take = [&](size_t nb) { char *r = q; q += align_up(nb); return r; };
    h.r = (double *)take((size_t)h.n * 8);
    h.rh = (double *)take((size_t)h.n * 8);
    h.p[0] = (double *)take((size_t)h.n * 8);
    h.p[1] = (double *)take((size_t)h.n * 8);
    h.v[0] = (double *)take((size_t)h.n * 8);
    h.v[1] = (double *)take((size_t)h.n * 8);
    h.t = (double *)take((size_t)h.n * 8);
    h.y = (double *)take((size_t)h.n * 8);
    for (int k = 0; k < 6; ++k) h.as[k] = (double *)take((size_t)h.n * 8);
    h.s1 = (double *)take((size_t)h.n * 8);
    h.t1 = (double *)take((size_t)h.n * 8);
    h.f = (double *)take((size_t)h.n * 8);
    h.dinv = (double *)take((size_t)h.n * 8);
    if (f32) {
        for (int k = 0; k < 4; ++k) h.sym32[k] = (float *)take((size_t)h.n * 4);
        for (int k = 0; k < 6; ++k) h.as32[k] = (float *)take((size_t)h.n * 4);
        h.r32 = (float *)take((size_t)h.n * 4);
        h.rh32 = (float *)take((size_t)h.n * 4);
        h.p32[0] = (float *)take((size_t)h.n * 4);
        h.p32[1] = (float *)take((size_t)h.n * 4);
        h.v32[0] = (float *)take((size_t)h.n * 4);
        h.v32[1] = (float *)take((size_t)h.n * 4);
        h.t32 = (float *)take((size_t)h.n * 4);
        h.d32 = (float *)take((size_t)h.n * 4);
        h.s1_32 = (float *)take((size_t)h.n * 4);
        h.t1_32 = (float *)take((size_t)h.n * 4);
        h.f32 = (float *)take((size_t)h.n * 4);
    }
    h.partials = (double *)take(partial_rows * kMaxRed * 8);
    h.counter = (uint32_t *)take(kAlign);
    h.last_iters = -1;
}

void fill_desc(eqs_ctx *c, int s) {
    SetHost &h = c->sets[s];
    SetDesc &d = c->h_desc[s];
    d.nx = h.g.nx;
    d.ny = h.g.ny;
    d.nz = h.g.nz;
    d.plane = h.plane;
    d.n = h.n;
    d.S = h.S;
    d.KC = h.KC;
    d.NKC = h.NKC;
    d.ntiles = h.ntiles;
    d.nflat = h.nflat;
    d.fS = h.fS;
    d.fntiles = h.fntiles;
    d.ford = h.ford;
    d.r = h.r;
    d.rh = h.rh;
    d.p[0] = h.p[0];
    d.p[1] = h.p[1];
    d.v[0] = h.v[0];
    d.v[1] = h.v[1];
    d.t = h.t;
    d.y = h.y;
    d.s1 = h.s1;
    d.t1 = h.t1;
    d.f = h.f;
    for (int k = 0; k < 6; ++k) d.as[k] = h.as[k];
    for (int k = 0; k < 6; ++k) d.as32[k] = h.as32[k];
    d.dinv = h.dinv;
    for (int k = 0; k < 4; ++k) d.sym32[k] = h.sym32[k];
    d.r32 = h.r32;
    d.rh32 = h.rh32;
    d.p32[0] = h.p32[0];
    d.p32[1] = h.p32[1];
    d.v32[0] = h.v32[0];
    d.v32[1] = h.v32[1];
    d.t32 = h.t32;
    d.d32 = h.d32;
    d.s1_32 = h.s1_32;
    d.t1_32 = h.t1_32;
    d.f32 = h.f32;
    d.partials = h.partials;
    d.counter = h.counter;
    d.st = c->d_state + s;
    d.sigma_tol[0] = sigma_tol(false);
    d.sigma_tol[1] = sigma_tol(true);
    d.sig_redo = env_int("EQS_SIGMA_REDO", 0) != 0 ? 1 : 0;
    const bool mg = c->d_mg && s < (int)c->mg.size() && !c->mg[s].empty();
    d.mg = mg ? c->d_mg + (size_t)s * kMgMaxLevels : nullptr;
    d.mg_levels = mg ? (int)c->mg[s].size() : 0;
}

LaunchSets launch_table(eqs_ctx *c, int first, int count, int *total, int *total_flat) {
    LaunchSets ls;
    memset(&ls, 0, sizeof(ls));
    ls.nsets = count;
    int acc = 0, accf = 0, accu = 0;
    for (int i = 0; i < count; ++i) {
        ls.tile_begin[i] = acc;
        ls.flat_begin[i] = accf;
        ls.ftile_begin[i] = accu;
        acc += c->sets[first + i].ntiles;
        accf += c->sets[first + i].nflat;
        accu += c->sets[first + i].fntiles;
    }
    for (int i = count; i <= kMaxSets; ++i) {
        ls.tile_begin[i] = acc;
        ls.flat_begin[i] = accf;
        ls.ftile_begin[i] = accu;
    }
    ls.fnt = c->fnt;
    ls.desc = c->d_desc + first;
    // each XCD runs a share of every set ($EQS_XBAL=0: one contiguous run of the launch per XCD)
    ls.xbal = env_int("EQS_XBAL", 1) != 0 ? 7 : 0;
    *total = acc;
    *total_flat = accf;
    return ls;
}

struct Run {
    eqs_ctx *c;
    int first, count;
    LaunchSets ls;
    int ntiles, nflat;
    int max_nx;
    bool fp32, trans;
    bool sym = false;   // every set exactly symmetric: the symmetric form of the single-sync step
    bool raw = false;   // the raw form of the single-sync step (FP64 forward solves, asked for on the context)
    int form() const { return raw ? 2 : (sym ? 1 : 0); }  // the step's form (kForm* of the kernels)
    long guard_limit;

    int L(Kern k, const double *x = nullptr, double *y = nullptr, int arg = 0, bool f32 = false) {
        c->launches++;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const int kind = (int)k * 2 + (f32 ? 1 : 0);
        const int pos = c->kpos[kind]++;
        const bool timed = ((c->profile_mask >> (int)k) & 1u) && (c->kseen[kind]++ % c->profile_every == 0);
        if (timed) {
            while (c->ev_pool.size() < c->ev_used + 2) {
                hipEvent_t e;
                EQS_HIP(hipEventCreate(&e));
                c->ev_pool.push_back(e);
            }
            e0 = c->ev_pool[c->ev_used];
            e1 = c->ev_pool[c->ev_used + 1];
            c->ev_used += 2;
            c->ev_kind.push_back(kind);
            c->ev_pos.push_back(pos);
        }
        // a timed launch carries the events itself: they take the kernel's own start and end
        if (launch_kernel(k, ls, ntiles, nflat, c->cpt, max_nx, f32, trans, c->stream, x, y, arg, e0, e1) !=
            hipSuccess) {
            (void)hipGetLastError();
            c->broken = true;
            return EQS_ERR_HIP;
        }
        return 0;
    }
    int readback() {
        c->readbacks++;
        int before = 0;
        for (int i = 0; i < count; ++i) before = std::max(before, (int)c->h_state[first + i].iters);
        EQS_HIP(hipMemcpyAsync(c->h_state + first, c->d_state + first, sizeof(SolveState) * count,
                               hipMemcpyDeviceToHost, c->stream));
        EQS_HIP(hipStreamSynchronize(c->stream));
        if (c->trace) {
            for (int i = 0; i < count; ++i) {
                const SolveState &q = c->h_state[first + i];
                fprintf(stderr, "eqsolve trace set %d: iters %d outer %d active %d done %d status %d |r| %.3e lim %.3e true %.3e\n",
                        first + i, q.iters, q.outer, q.active, q.done, q.status, sqrt(q.rr), q.lim2, sqrt(q.rr_true));
            }
        }
        if (c->profile_mask) {
            // A set that stops iterating stays stopped until the host acts, so
            // of the iteration launches since the last look, the first
            // (iterations done) did work and the rest exited at once: only
            // the former enter the per-kernel means.
            int after = 0;
            for (int i = 0; i < count; ++i) after = std::max(after, (int)c->h_state[first + i].iters);
            const int worked = std::max(0, after - before);
            for (size_t i = 0; i < c->ev_kind.size(); ++i) {
                const int kind = c->ev_kind[i];
                const int kk = kind / 2;
                const bool iter_kernel = kk == K_K1 || kk == K_K2 || kk == K_K3 || kk == K_FUSED;
                if (iter_kernel && c->ev_pos[i] >= worked) continue;
                float ms = 0.f;
                EQS_HIP(hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
                c->kcount[kind]++;
                c->kms[kind] += ms;
            }
            c->ev_kind.clear();
            c->ev_pos.clear();
            c->ev_used = 0;
        }
        for (int i = 0; i < 2 * 32; ++i) c->kpos[i] = 0;
        return 0;
    }
    // C BiCGSTAB iterations (K1, K2, K3 each): replayed from captured graphs of
    // 2^k iterations (the launch table and the set table's device address
    // are fixed per context, so a graph stays valid across calls), or
    // launched one by one when per-launch timing is on.
    // hk: after every step, the refinement's per-set housekeeping (form the inner iterate, update x,
    // the FP64 residual, f = M^T r^ for the next inner solve), each launch doing work only for the
    // sets whose state asks for it, so a set whose inner solve ends starts its next one at once
    // instead of waiting for the others (FP32 forms, single-sync iteration)
    int iterate(int C, bool f32, bool hk = false) {
        int rc;
        auto housekeeping = [&](hipStream_t s) {
            bool ok = launch_kernel(K_MAT, ls, ntiles, nflat, c->cpt, max_nx, true, trans, s, nullptr, nullptr, 0) ==
                      hipSuccess;
            ok = ok && launch_kernel(K_UPDATE, ls, ntiles, nflat, c->cpt, max_nx, false, trans, s, nullptr, nullptr,
                                     0) == hipSuccess;
            ok = ok && launch_kernel(K_OUTER, ls, ntiles, nflat, c->cpt, max_nx, false, trans, s, nullptr, nullptr,
                                     0) == hipSuccess;
            ok = ok && launch_kernel(K_FSETUP, ls, ntiles, nflat, c->cpt, max_nx, true, trans, s, nullptr, nullptr,
                                     0) == hipSuccess;
            return ok;
        };
        if (c->profile_mask || !c->use_graphs) {
            for (int i = 0; i < C; ++i) {
                if (c->sync1) {
                    if ((rc = L(K_FUSED, nullptr, nullptr, form(), f32))) return rc;
                    if (hk) {
                        if ((rc = L(K_MAT, nullptr, nullptr, 0, true))) return rc;
                        if ((rc = L(K_UPDATE))) return rc;
                        if ((rc = L(K_OUTER))) return rc;
                        if ((rc = L(K_FSETUP, nullptr, nullptr, 0, true))) return rc;
                    }
                    continue;
                }
                if ((rc = L(K_K1, nullptr, nullptr, 0, f32))) return rc;
                if ((rc = L(K_K2, nullptr, nullptr, 0, f32))) return rc;
                if ((rc = L(K_K3, nullptr, nullptr, 0, f32))) return rc;
            }
            return 0;
        }
        const int per_iter = c->sync1 ? (hk ? 5 : 1) : 3;
        auto &slots = c->graphs[std::make_tuple(first, count, trans, f32, (c->sync1 ? form() : 0) + (hk ? 8 : 0))];
        for (int b = 8; b >= 0; --b) {
            while (C >= (1 << b)) {
                if (!slots[b]) {
                    if (!c->capture_stream) EQS_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
                    EQS_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
                    bool ok = true;
                    for (int i = 0; i < (1 << b) && ok; ++i) {
                        if (c->sync1) {
                            ok = launch_kernel(K_FUSED, ls, ntiles, nflat, c->cpt, max_nx, f32, trans,
                                               c->capture_stream, nullptr, nullptr, form()) == hipSuccess;
                            if (hk) ok = ok && housekeeping(c->capture_stream);
                            continue;
                        }
                        for (Kern k : {K_K1, K_K2, K_K3})
                            ok = ok && launch_kernel(k, ls, ntiles, nflat, c->cpt, max_nx, f32, trans,
                                                     c->capture_stream, nullptr, nullptr, 0) == hipSuccess;
                    }
                    hipGraph_t g = nullptr;
                    const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
                    if (!ok || e != hipSuccess || !g) {
                        if (g) (void)hipGraphDestroy(g);
                        (void)hipGetLastError();
                        c->broken = true;
                        return EQS_ERR_HIP;
                    }
                    hipGraphExec_t ex = nullptr;
                    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    if (ei != hipSuccess) {
                        (void)hipGetLastError();
                        c->broken = true;
                        return EQS_ERR_HIP;
                    }
                    slots[b] = ex;
                }
                EQS_HIP(hipGraphLaunch(slots[b], c->stream));
                c->launches += (uint64_t)per_iter << b;
                C -= 1 << b;
            }
        }
        return 0;
    }
    const SolveState &st(int i) const { return c->h_state[first + i]; }
    // after the setup's readback: the symmetric form when every set of the run takes it
    void pick_form() {
        sym = !raw && count > 0 && c->sync1;
        for (int i = 0; i < count; ++i) sym = sym && st(i).sym != 0;
        for (int i = 0; i < count; ++i) {
            c->sets[first + i].form_sym = sym;
            c->sets[first + i].form_raw = raw;
        }
    }
    bool all_done() const {
        for (int i = 0; i < count; ++i)
            if (!st(i).done) return false;
        return true;
    }
    template <class F>
    bool any(F f) const {
        for (int i = 0; i < count; ++i)
            if (f(st(i))) return true;
        return false;
    }
    void reset_rate() {
        for (int i = 0; i < count; ++i) c->sets[first + i].last_iters = -1;
    }
    // iterations to enqueue before the next look at the state
    int chunk() {
        int best = 2;
        bool any_active = false;
        for (int i = 0; i < count; ++i) {
            const SolveState &s = st(i);
            SetHost &h = c->sets[first + i];
            if (!s.active) continue;
            any_active = true;
            const double lrr = s.rr > 0 ? log(s.rr) : -700.0;
            const double lgoal = s.lim2 > 0 ? 2.0 * log(s.lim2) : -700.0;
            int want;
            if (h.last_iters >= 0 && s.iters > h.last_iters && lrr < h.last_log_rr) {
                const double slope = (lrr - h.last_log_rr) / (double)(s.iters - h.last_iters);
                const double rem = (lgoal - lrr) / slope;
                // BiCGSTAB residuals plateau and drop, so aim short of the
                // prediction and never more than double the last chunk
                want = (int)std::min(1e6, ceil(0.8 * std::max(0.0, rem))) + 1;
                const int prev = std::max(8, s.iters - h.last_iters);
                want = std::min(want, 2 * prev);
            } else {
                want = h.last_iters < 0 ? 8 : std::max(8, s.iters - std::max(0, h.last_iters));
            }
            h.last_iters = s.iters;
            h.last_log_rr = lrr;
            want = std::min(want, s.maxit - s.iters);
            best = std::max(best, want);
        }
        if (!any_active) return 0;
        return std::min(best, 1024);
    }
};

int run_fp64_mg(Run &R);
Run make_run(eqs_ctx *c, int first, int count, bool trans);

int run_fp64(Run &R) {
    int rc;
    // FP64 solves with the multigrid preconditioner: all the run's sets together
    if (R.c->precond == EQS_PRECOND_MG && !R.trans) return run_fp64_mg(R);
    // tiny sets: the whole solve in one launch, one block per set
    int max_n = 0;
    for (int i = 0; i < R.count; ++i) max_n = std::max(max_n, R.c->sets[R.first + i].n);
    if (max_n <= kSmallSolveMaxCells && R.c->use_small) {
        R.c->launches++;
        if (launch_small(R.ls, max_n, R.trans, R.c->stream) != hipSuccess) {
            (void)hipGetLastError();
            R.c->broken = true;
            return EQS_ERR_HIP;
        }
        return R.readback();
    }
    const bool s1 = R.c->sync1;
    // the raw form needs no per-solve coefficients: the setup pass writes 1/a_P
    R.raw = s1 && !R.trans && R.c->step_form == EQS_STEP_UNSCALED;
    // coefficients of A D^-1 (A^T D^-1) and 1/a_P, once per solve; symmetry check
    if (!R.raw && (rc = R.L(K_SCALE, nullptr, nullptr, R.c->sym_on))) return rc;
    if ((rc = R.L(K_SETUP, nullptr, nullptr, R.raw ? 1 : 0))) return rc;
    if (s1 && (rc = R.L(K_FSETUP, nullptr, nullptr, R.raw ? 2 : 0))) return rc;
    if ((rc = R.readback())) return rc;
    R.pick_form();
    R.reset_rate();
    for (long guard = 0;; ++guard) {
        if (guard > R.guard_limit) { R.c->broken = true; return EQS_ERR_STATE; }
        if (R.all_done()) break;
        if (R.any([s1](const SolveState &s) {
                return !s.done && (s.converged || s.need_report || (s1 && (s.mat || s.need_f)));
            })) {
            if (s1 && (rc = R.L(K_MAT))) return rc;  // the iterate of the step being left
            if ((rc = R.L(K_UNSCALE))) return rc;  // x = y / a_P
            if ((rc = R.L(K_RECHECK))) return rc;
            if ((rc = R.L(K_REPORT))) return rc;
            if (s1 && (rc = R.L(K_FSETUP, nullptr, nullptr, R.raw ? 2 : 0))) return rc;  // after a restart
            if ((rc = R.readback())) return rc;
            R.reset_rate();
            continue;
        }
        const int C = R.chunk();
        if (C <= 0) { R.c->broken = true; return EQS_ERR_STATE; }
        if ((rc = R.iterate(C, false))) return rc;
        if ((rc = R.readback())) return rc;
    }
    if (R.any([](const SolveState &s) { return s.zero_rhs != 0; }))
        if ((rc = R.L(K_ZERO, nullptr, nullptr, 0))) return rc;
    return 0;
}

int run_fp32(Run &R) {
    int rc;
    const bool s1 = R.c->sync1;
    if ((rc = R.L(K_CAST, nullptr, nullptr, R.c->sym_on))) return rc;
    if ((rc = R.L(K_OUTER))) return rc;
    if (s1 && (rc = R.L(K_FSETUP, nullptr, nullptr, 0, true))) return rc;
    if ((rc = R.readback())) return rc;
    R.pick_form();
    R.reset_rate();
    // A batch of large sets runs the refinement's housekeeping in the launch stream after every
    // step (EQS_REFINE_INSTREAM=0: between chunks, when the host sees a set's inner solve end), so no
    // set idles while the others finish their inner solves.  Small sets keep the host-driven
    // rounds: there the extra launches would cost more than a step.
    long cells = 0;
    for (int i = 0; i < R.count; ++i) cells += R.c->sets[R.first + i].n;
    const bool hk = s1 && R.count > 1 && env_int("EQS_REFINE_INSTREAM", 1) != 0 &&
                    cells >= env_int("EQS_REFINE_INSTREAM_CELLS", 1 << 22);
    for (long guard = 0;; ++guard) {
        if (guard > R.guard_limit) { R.c->broken = true; return EQS_ERR_STATE; }
        if (R.all_done()) break;
        if (hk) {
            // every housekeeping step is already in the stream: look at the state every 16 steps
            if ((rc = R.iterate(16, true, true))) return rc;
            if ((rc = R.readback())) return rc;
            continue;
        }
        if (R.any([s1](const SolveState &s) {
                return !s.done && (s.inner_done != 0 || (s1 && (s.mat || s.need_f)));
            })) {
            if (s1 && (rc = R.L(K_MAT, nullptr, nullptr, 0, true))) return rc;
            if ((rc = R.L(K_UPDATE))) return rc;
            if ((rc = R.L(K_OUTER))) return rc;
            if (s1 && (rc = R.L(K_FSETUP, nullptr, nullptr, 0, true))) return rc;
            if ((rc = R.readback())) return rc;
            R.reset_rate();
            continue;
        }
        const int C = R.chunk();
        if (C <= 0) { R.c->broken = true; return EQS_ERR_STATE; }
        if ((rc = R.iterate(C, true))) return rc;
        if ((rc = R.readback())) return rc;
    }
    if (R.any([](const SolveState &s) { return s.zero_rhs != 0; }))
        if ((rc = R.L(K_ZERO, nullptr, nullptr, 0))) return rc;
    return 0;
}

Run make_run(eqs_ctx *c, int first, int count, bool trans) {
    Run R;
    R.c = c;
    R.first = first;
    R.count = count;
    R.ls = launch_table(c, first, count, &R.ntiles, &R.nflat);
    R.max_nx = 1;
    for (int i = 0; i < count; ++i) R.max_nx = std::max(R.max_nx, c->sets[first + i].g.nx);
    R.fp32 = false;
    R.trans = trans;
    for (int i = 0; i < count; ++i) c->sets[first + i].form_sym = c->sets[first + i].form_raw = false;
    // every host loop turn either runs >= 1 iteration or one housekeeping
    // step that only follows an iteration, so 2*maxit + slack turns suffice
    long mx = 0;
    for (int i = 0; i < count; ++i) mx = std::max<long>(mx, c->h_desc[first + i].maxit);
    R.guard_limit = 2 * mx + 64;
    return R;
}

void write_info(eqs_ctx *c, int s, eqs_info *info) {
    if (!info) return;
    const SolveState &st = c->h_state[s];
    info->status = st.status;
    info->iters = st.iters;
    info->outer = (st.mode == MODE_REFINE || st.mode == MODE_FP32) ? st.outer : st.restarts;
    info->flags = (c->sets[s].form_sym ? EQS_INFO_SYMMETRIC : 0) | (c->sets[s].form_raw ? EQS_INFO_UNSCALED : 0);
    info->sigma_restarts = st.sig_restarts;
    info->sigma_reruns = st.sig_redos;
    if (st.zero_rhs)
        info->rel_res = 0.0;
    else if (st.bb_outer > 0)
        info->rel_res = sqrt(st.rr_true / st.bb_outer);
    else
        info->rel_res = NAN;
}

bool diag_ok(const double *const diag[7]) {
    if (!diag) return false;
    for (int k = 0; k < 7; ++k)
        if (!diag[k]) return false;
    return true;
}

bool aliases(const void *x, const double *const diag[7], const void *b) {
    if (x == b) return true;
    for (int k = 0; k < 7; ++k)
        if ((const void *)diag[k] == x) return true;
    return false;
}

int set_mode_for(int precision) {
    return precision == EQS_FP32_REFINE ? MODE_REFINE : (precision == EQS_FP32 ? MODE_FP32 : MODE_FP64);
}

int upload_desc(eqs_ctx *c, int first, int count) {
    EQS_HIP(hipMemcpyAsync(c->d_desc + first, c->h_desc + first, sizeof(SetDesc) * count, hipMemcpyHostToDevice,
                           c->stream));
    return 0;
}


// ------------------------------------------------------------------ tuning

std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

struct TuneEntry {
    int cpt, kc, nflat;
    int fnt, ford;  // the single-sync step's block size and tile order
    double us;
};

// JSON lines, one object per tuned (arch, grid, precision); the last match wins
bool cache_lookup(const char *path, const std::string &arch, const eqs_grid &g, int precision, TuneEntry *out) {
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512], a[64];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        int nx, ny, nz, pr, cpt, kc, nflat, fnt, ford;
        double us;
        if (sscanf(line,
                   "{\"arch\": \"%63[^\"]\", \"nx\": %d, \"ny\": %d, \"nz\": %d, \"precision\": %d, \"cpt\": %d, "
                   "\"kc\": %d, \"nflat\": %d, \"fnt\": %d, \"ford\": %d, \"us_per_iter\": %lf}",
                   a, &nx, &ny, &nz, &pr, &cpt, &kc, &nflat, &fnt, &ford, &us) == 11 &&
            arch == a && nx == g.nx && ny == g.ny && nz == g.nz && pr == precision && (cpt == 1 || cpt == 2) &&
            (fnt == 256 || fnt == 512) && (ford == 0 || ford == 1)) {
            *out = TuneEntry{cpt, kc, nflat, fnt, ford, us};
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &arch, const eqs_grid &g, int precision, const TuneEntry &e) {
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"arch\": \"%s\", \"nx\": %d, \"ny\": %d, \"nz\": %d, \"precision\": %d, \"cpt\": %d, \"kc\": %d, "
            "\"nflat\": %d, \"fnt\": %d, \"ford\": %d, \"us_per_iter\": %.3f}\n",
            arch.c_str(), g.nx, g.ny, g.nz, precision, e.cpt, e.kc, e.nflat, e.fnt, e.ford, e.us);
    fclose(f);
}

void clear_graphs(eqs_ctx *c) {
    for (auto &kv : c->graphs)
        for (hipGraphExec_t ex : kv.second)
            if (ex) (void)hipGraphExecDestroy(ex);
    c->graphs.clear();
    for (auto &kv : c->graphs_mg)
        for (hipGraphExec_t ex : kv.second)
            if (ex) (void)hipGraphExecDestroy(ex);
    c->graphs_mg.clear();
}

// ------------------------------------------------------------------ multigrid-preconditioned iteration

// z = B^-1 r for every set of the run: one V-cycle each, the sets sharing every launch (which: the
// input and output, see launch_mg_restrict); gated launches do nothing for a set that stopped
// iterating.  The finest level goes through the k-march on the run's tiles (the per-cell residual
// in each set's y buffer, unused by this iteration); the coarser levels through per-cell kernels
// that take the sets along blockIdx.y, a set doing its own levels in its own order (a set with fewer
// levels skips the launches of levels it does not have).
hipError_t mg_vcycle(const Run &R, int which, bool gated, hipStream_t stream) {
    eqs_ctx *c = R.c;
    int nl = 0;
    for (int i = 0; i < R.count; ++i) nl = std::max(nl, (int)c->mg[R.first + i].size());
    // the largest set's cells on level l among the sets that have level `upto` or more levels
    auto cells = [&](int l, int need) {
        int m = 1;
        for (int i = 0; i < R.count; ++i) {
            const std::vector<MgLevel> &L = c->mg[R.first + i];
            if ((int)L.size() >= need) m = std::max(m, L[l].n);
        }
        return m;
    };
    const SetDesc *dd = c->d_desc + R.first;
    const MgLevel *lv = c->d_mg + (size_t)R.first * kMgMaxLevels;
    const int ns = R.count;
    MgCounts cnt{};
    for (int i = 0; i < ns; ++i) cnt.n[i] = (int)c->mg[R.first + i].size();
    hipError_t e = hipSuccess;
    if (nl > 1) {
        e = launch_mg_fine(R.ls, lv, cnt, R.ntiles, c->cpt, R.max_nx, which, true, c->mgp, gated, stream);
        if (e == hipSuccess) e = launch_mg_aggregate(dd, lv, cnt, ns, cells(1, 2), gated, stream);
    }
    for (int l = 1; l + 1 < nl && e == hipSuccess; ++l)
        e = launch_mg_restrict(dd, lv, cnt, ns, l, cells(l + 1, l + 2), c->mgp, gated, stream);
    if (e == hipSuccess) e = launch_mg_coarsest(dd, lv, cnt, ns, which, c->mgp, gated, stream);
    for (int l = nl - 2; l >= 1 && e == hipSuccess; --l)
        e = launch_mg_prolong(dd, lv, cnt, ns, l, cells(l, l + 2), c->mgp, gated, stream);
    if (nl > 1 && e == hipSuccess)
        e = launch_mg_fine(R.ls, lv, cnt, R.ntiles, c->cpt, R.max_nx, which, false, c->mgp, gated, stream);
    c->launches += 2 * nl;
    return e;
}

// the Galerkin operators of every coarse level of set s, from the diagonals in its table entry
hipError_t mg_coarsen_all(eqs_ctx *c, int s) {
    const std::vector<MgLevel> &L = c->mg[s];
    // exact symmetry of this call's matrix (EQS_MG_SYM=0: never assumed)
    hipError_t e = launch_mg_symcheck(c->d_desc + s, L[0].n, env_int("EQS_MG_SYM", 1) != 0, c->stream);
    if (e == hipSuccess) e = launch_mg_round0(c->d_desc + s, c->d_mg + (size_t)s * kMgMaxLevels, L[0].n, c->stream);
    for (int l = 0; l + 1 < (int)L.size() && e == hipSuccess; ++l)
        e = launch_mg_coarsen(c->d_desc + s, c->d_mg + (size_t)s * kMgMaxLevels, l, L[l + 1].n, c->stream);
    return e;
}

// one preconditioned BiCGSTAB iteration of the run's sets on `stream`
hipError_t mg_iteration(Run &R, hipStream_t stream) {
    eqs_ctx *c = R.c;
    auto K = [&](Kern k) {
        c->launches++;
        return launch_kernel(k, R.ls, R.ntiles, R.nflat, c->cpt, R.max_nx, false, false, stream, nullptr, nullptr, 0);
    };
    hipError_t e = K(K_PC_P);
    if (e == hipSuccess) e = mg_vcycle(R, 0, true, stream);  // p^ = B^-1 p
    if (e == hipSuccess) e = K(K_PC_V);
    // s = r - alpha v: the s-cycle's residual pass forms it for sets with a finest-level pass; the
    // pointwise kernel only for single-level sets
    bool single = false;
    for (int i = 0; i < R.count; ++i) single = single || c->mg[R.first + i].size() < 2;
    if (e == hipSuccess && single) e = K(K_PC_S);
    if (e == hipSuccess) e = mg_vcycle(R, 1, true, stream);  // s^ = B^-1 s
    if (e == hipSuccess) e = K(K_PC_T);
    if (e == hipSuccess) e = K(K_PC_X);
    return e;
}

// C iterations: replayed from captured graphs of 1, 2, 4 or 8 iterations (launched one
// by one when graphs are off)
int mg_iterate(Run &R, int C) {
    eqs_ctx *c = R.c;
    if (!c->use_graphs) {
        for (int i = 0; i < C; ++i)
            if (mg_iteration(R, c->stream) != hipSuccess) {
                (void)hipGetLastError();
                c->broken = true;
                return EQS_ERR_HIP;
            }
        return 0;
    }
    auto &slots = c->graphs_mg[std::make_pair(R.first, R.count)];
    for (int b = 3; b >= 0; --b) {
        while (C >= (1 << b)) {
            if (!slots[b]) {
                if (!c->capture_stream) EQS_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
                EQS_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
                bool ok = true;
                const uint64_t before = c->launches;
                for (int i = 0; i < (1 << b) && ok; ++i) ok = mg_iteration(R, c->capture_stream) == hipSuccess;
                c->launches = before;
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
                hipGraphExec_t ex = nullptr;
                const hipError_t ei = (ok && e == hipSuccess && g) ? hipGraphInstantiate(&ex, g, nullptr, nullptr, 0)
                                                                   : hipErrorUnknown;
                if (g) (void)hipGraphDestroy(g);
                if (ei != hipSuccess) {
                    (void)hipGetLastError();
                    c->broken = true;
                    return EQS_ERR_HIP;
                }
                slots[b] = ex;
            }
            EQS_HIP(hipGraphLaunch(slots[b], c->stream));
            c->launches += (uint64_t)(5 + 2 * (2 * (int)c->mg[R.first].size())) << b;  // (first set's count)
            C -= 1 << b;
        }
    }
    return 0;
}

int run_fp64_mg(Run &R) {
    int rc;
    for (int i = 0; i < R.count; ++i) {
        if (mg_coarsen_all(R.c, R.first + i) != hipSuccess) {
            (void)hipGetLastError();
            R.c->broken = true;
            return EQS_ERR_HIP;
        }
        R.c->launches += R.c->mg[R.first + i].size();
    }
    if ((rc = R.L(K_SETUP))) return rc;
    if ((rc = R.readback())) return rc;
    R.reset_rate();
    for (long guard = 0;; ++guard) {
        if (guard > R.guard_limit) { R.c->broken = true; return EQS_ERR_STATE; }
        if (R.all_done()) break;
        if (R.any([](const SolveState &s) { return s.converged || s.need_report; })) {
            if ((rc = R.L(K_RECHECK))) return rc;  // x is updated in place: no unscaling
            if ((rc = R.L(K_REPORT))) return rc;
            if ((rc = R.readback())) return rc;
            R.reset_rate();
            continue;
        }
        const int C = std::min(R.chunk(), 15);
        if (C <= 0) { R.c->broken = true; return EQS_ERR_STATE; }
        if ((rc = mg_iterate(R, C))) return rc;
        if ((rc = R.readback())) return rc;
    }
    if (R.any([](const SolveState &s) { return s.zero_rhs != 0; }))
        if ((rc = R.L(K_ZERO, nullptr, nullptr, 0))) return rc;
    return 0;
}

// Mean time of one BiCGSTAB iteration (K1 + K2 + K3, or the fused step) of sets
// [first, first + count) in one launch table under their current tilings, every set on the
// synthetic system held in `tmp` (7 diagonals, b, x, each `stride` cells apart; a set reads
// its first n cells, and nothing the timed kernels write aliases them).  Returns -1 on a HIP
// failure and -2 if the measurement is not a full-work timing (a set stopped iterating
// meanwhile).  The general form of the step is timed (the synthetic system is symmetric).
double time_steps(eqs_ctx *c, int first, int count, double *tmp, size_t stride, int iters) {
    const bool f32 = c->precision != EQS_FP64;
    for (int s = first; s < first + count; ++s) {
        fill_desc(c, s);
        SetDesc &d = c->h_desc[s];
        for (int k = 0; k < 7; ++k) d.a[k] = tmp + k * stride;
        d.b = tmp + 7 * stride;
        d.x = tmp + 8 * stride;
        d.xf = nullptr;
        for (int k = 0; k < 7; ++k) d.g[k] = nullptr;
        d.mode = f32 ? MODE_REFINE : MODE_FP64;
        d.tol = 1e-15;
        d.tol_inner = 1e-15;
        d.maxit = 1 << 30;
    }
    if (upload_desc(c, first, count)) return -1.0;
    if (launch_fill(tmp + 8 * stride, (long)stride, 0.0, c->stream) != hipSuccess) return -1.0;
    Run R = make_run(c, first, count, false);
    const int saved = c->profile_mask;
    c->profile_mask = 0;
    if (f32) {
        if (R.L(K_CAST) || R.L(K_OUTER)) return -1.0;
    } else if (R.L(K_SCALE) || R.L(K_SETUP)) {
        return -1.0;
    }
    if (c->sync1 && R.L(K_FSETUP, nullptr, nullptr, 0, f32)) return -1.0;
    auto step = [&]() -> int {
        if (c->sync1) return R.L(K_FUSED, nullptr, nullptr, 0, f32);
        for (Kern k : {K_K1, K_K2, K_K3})
            if (int rc = R.L(k, nullptr, nullptr, 0, f32)) return rc;
        return 0;
    };
    for (int i = 0; i < 2; ++i)
        if (step()) return -1.0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    (void)hipEventRecord(e0, c->stream);
    for (int i = 0; i < iters; ++i)
        if (step()) return -1.0;
    (void)hipEventRecord(e1, c->stream);
    float ms = 0.f;
    const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->profile_mask = saved;
    if (!ok || R.readback()) return -1.0;
    for (int s = first; s < first + count; ++s)
        if (!c->h_state[s].active) return -2.0;
    return 1e3 * ms / iters;
}

// planes per chunk of a multigrid-preconditioned solve: its fine-level passes stream few
// operands per step, so they need more blocks in flight than the fused Jacobi step (measured on
// the 128x256x128 pressure-like system, 2 cells per thread: 32 planes 12.3 ms per solve, 16 planes
// 10.5, 8 planes 9.7, 4 planes 9.9)
int mg_kc() { return std::max(1, env_int("EQS_MG_KC", 8)); }

// the tiling for the selected preconditioner: the Jacobi iteration's own depth, or at most
// mg_kc() planes per chunk under multigrid
void retile_for_precond(eqs_ctx *c) {
    for (int s = 0; s < c->nsets; ++s) {
        SetHost &h = c->sets[s];
        if (h.kc_jacobi <= 0) h.kc_jacobi = h.KC;
        const int kc = c->precond == EQS_PRECOND_MG ? std::min(mg_kc(), h.kc_jacobi) : h.kc_jacobi;
        set_tiling(h, c->cpt, kc, h.nflat, c->fnt, h.ford);
        fill_desc(c, s);
    }
}

int apply_tuning(eqs_ctx *c, int cpt, int fnt, const std::vector<TuneEntry> &e) {
    c->cpt = cpt;
    c->fnt = fnt;
    for (int s = 0; s < c->nsets; ++s) {
        set_tiling(c->sets[s], cpt, e[s].kc, e[s].nflat, fnt, e[s].ford);
        c->sets[s].kc_jacobi = c->sets[s].KC;
        fill_desc(c, s);
    }
    retile_for_precond(c);
    clear_graphs(c);
    return upload_desc(c, 0, c->nsets);
}

// The iteration scheme (c->sync1, c->sym_on) and cells per thread of a context for these grids,
// before any tuning: the single-sync iteration (EQS_SYNC=3 selects the three-launch one) where
// its wider planes fit in LDS, with the narrower segment if need be.  Returns the cells per
// thread, or -1 if nx is beyond what one LDS plane buffer or the halo slots cover.
int default_shape(eqs_ctx *c, const eqs_grid *grids, int nsets, int *max_nx_out) {
    int max_nx = 1;
    long long max_plane = 1;
    for (int s = 0; s < nsets; ++s) {
        max_nx = std::max(max_nx, grids[s].nx);
        max_plane = std::max(max_plane, (long long)grids[s].nx * grids[s].ny);
    }
    int cpt = env_int("EQS_CPT", 0);
    if (cpt != 1 && cpt != 2) cpt = max_plane >= 4 * kBlock ? 2 : 1;
    while (cpt > 1 && march_lds_bytes(cpt, max_nx, 8) > kMaxLds) cpt /= 2;
    c->sym_on = env_int("EQS_SYM", 1) != 0 ? 1 : 0;
    // the single-sync step in blocks of 256 threads, or 512 where EQS_FNT=512 asks for it and the
    // shape has that instantiation (the tuner chooses between them by measurement)
    auto fits = [&](int fc, int nt) {
        return fused_shape_ok(fc, max_nx, nt) && fused_lds_bytes(fc, max_nx, 8, nt) <= c->fused_lds_cap;
    };
    int fnt = env_int("EQS_FNT", 256) == 512 ? 512 : 256;
    if (fnt == 512 && !fits(cpt, 512)) fnt = 256;
    c->sync1 = env_int("EQS_SYNC", 1) != 3;
    if (c->sync1) {
        int fc = cpt;
        while (fc > 1 && !fits(fc, fnt)) fc /= 2;
        if (!fits(fc, fnt))
            c->sync1 = false;
        else
            cpt = fc;
    }
    c->fnt = c->sync1 ? fnt : 256;
    *max_nx_out = max_nx;
    if (march_lds_bytes(cpt, max_nx, 8) > kMaxLds || halo_slots(max_nx, kBlock) < 0) return -1;
    return cpt;
}

// ------------------------------------------------------------------ solve on a static workspace
//
// One FP64 set solved on a workspace the caller lends (eqsolve_solve_noalloc's static device
// array): the context, its set table and its state block live in static host memory, one per
// device, and every device-side array is carved out of the workspace, so nothing is allocated
// on the host or the device.  Iteration chunks are launched one by one (no graphs).

constexpr int kStaticDevices = 64;
eqs_ctx g_static_ctx[kStaticDevices];
SetDesc g_static_desc[kStaticDevices];
SolveState g_static_state[kStaticDevices];

}  // namespace

namespace eqs {

size_t static_solve_bytes(const eqs_grid &g) {
    eqs_ctx probe;  // shape only: no allocation, no HIP call (64 KB of LDS per block at most)
    probe.nsets = 1;
    int max_nx = 1;
    const int cpt = default_shape(&probe, &g, 1, &max_nx);
    if (cpt < 0) return 0;
    SetHost h{};
    h.g = g;
    h.plane = g.nx * g.ny;
    h.n = h.plane * g.nz;
    choose_tiling(h, cpt, probe.fnt);
    return align_up(sizeof(SetDesc)) + align_up(sizeof(SolveState)) +
           set_ws_bytes(h, false, (size_t)std::max(h.ntiles, h.nflat));
}

int static_solve(void *ws, size_t cap, int device, const eqs_grid &g, const double *const diag[7], const double *b,
                 double *x, double tol, int32_t maxit, eqs_info *info, void *hip_stream) {
    if (device < 0 || device >= kStaticDevices || !ws) return EQS_ERR_STATE;
    const size_t need = static_solve_bytes(g);
    if (need == 0) return EQS_ERR_ARG;
    if (need > cap) return EQS_ERR_SIZE;
    eqs_ctx *c = &g_static_ctx[device];
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->nsets = 1;
    c->precision = EQS_FP64;
    c->trace = env_int("EQS_TRACE", 0) != 0;
    c->use_graphs = false;
    c->use_small = env_int("EQS_SMALL", 1) != 0;
    c->broken = false;
    c->profile_mask = 0;
    c->precond = EQS_PRECOND_JACOBI;
    c->fused_lds_cap = kMaxLds;
    int max_nx = 1;
    c->cpt = default_shape(c, &g, 1, &max_nx);
    c->max_nx = max_nx;
    SetHost &h = c->sets[0];
    memset(&h, 0, sizeof(h));
    h.g = g;
    h.plane = g.nx * g.ny;
    h.n = h.plane * g.nz;
    choose_tiling(h, c->cpt, c->fnt);
    char *w = (char *)ws;
    c->d_desc = (SetDesc *)w;
    c->d_state = (SolveState *)(w + align_up(sizeof(SetDesc)));
    c->h_desc = &g_static_desc[device];
    c->h_state = &g_static_state[device];
    c->ws = w + align_up(sizeof(SetDesc)) + align_up(sizeof(SolveState));
    c->ws_bytes = need - align_up(sizeof(SetDesc)) - align_up(sizeof(SolveState));
    carve_set(h, (char *)c->ws, false, (size_t)std::max(h.ntiles, h.nflat));
    memset(c->h_desc, 0, sizeof(SetDesc));
    memset(c->h_state, 0, sizeof(SolveState));
    fill_desc(c, 0);
    SetDesc &d = c->h_desc[0];
    for (int k = 0; k < 7; ++k) d.a[k] = diag[k];
    d.b = b;
    d.x = x;
    d.mode = MODE_FP64;
    d.tol = tol;
    d.tol_inner = inner_tol();
    d.maxit = maxit;
    // The array keeps the previous call's contents: clear all of this call's part (the state
    // block, the ticket counter, every vector) with a fill kernel, then upload the set table.
    if (launch_fill((double *)w, (long)(need / sizeof(double)), 0.0, c->stream) != hipSuccess) {
        (void)hipGetLastError();
        return EQS_ERR_HIP;
    }
    int rc = upload_desc(c, 0, 1);
    if (rc) return rc;
    Run R = make_run(c, 0, 1, false);
    if ((rc = run_fp64(R))) return rc;
    if ((rc = R.readback())) return rc;
    write_info(c, 0, info);
    return c->h_state[0].status;
}

}  // namespace eqs

namespace {
}  // namespace

extern "C" {

int eqsolve_create(eqs_ctx **out, const eqs_grid *grids, int32_t nsets, int32_t precision, void *hip_stream) {
    if (!out) return EQS_ERR_ARG;
    *out = nullptr;
    if (!grids || nsets < 1 || nsets > kMaxSets) return EQS_ERR_ARG;
    if (precision != EQS_FP64 && precision != EQS_FP32_REFINE && precision != EQS_FP32) return EQS_ERR_ARG;
    for (int s = 0; s < nsets; ++s)
        if (!grid_ok(grids[s])) return EQS_ERR_ARG;

    eqs_ctx *c = new (std::nothrow) eqs_ctx();
    if (!c) return EQS_ERR_NOMEM;
    c->stream = (hipStream_t)hip_stream;
    c->trace = env_int("EQS_TRACE", 0) != 0;
    c->use_graphs = env_int("EQS_GRAPHS", 1) != 0;
    c->use_small = env_int("EQS_SMALL", 1) != 0;
    c->nsets = nsets;
    c->precision = precision;
    c->step_form = precision == EQS_FP64 && env_int("EQS_UNSCALED", 0) != 0 ? EQS_STEP_UNSCALED : EQS_STEP_SCALED;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return EQS_ERR_HIP; }
    // the single-sync step may take the device's whole per-block LDS (160 KB on gfx950; the march
    // kernels stay within 64 KB); EQS_FUSED_LDS caps it for tests
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
            (void)hipGetLastError();
            lds = (int)kMaxLds;
        }
        // (less 1 KB: the kernels' static LDS, the reduction scratch, counts against the same limit)
        size_t cap = (size_t)std::max<long>((long)kMaxLds, std::min<long>((long)lds, 160L * 1024) - 1024);
        cap = std::min(cap, (size_t)std::max(env_int("EQS_FUSED_LDS", (int)cap), (int)kMaxLds));
        if (cap > kMaxLds && allow_fused_lds(cap) != hipSuccess) {
            (void)hipGetLastError();
            cap = kMaxLds;
        }
        c->fused_lds_cap = cap;
    }

    int max_nx = 1;
    int cpt = default_shape(c, grids, nsets, &max_nx);
    if (cpt < 0) { delete c; return EQS_ERR_ARG; }
    // a tuning cache (EQS_TUNE_CACHE) entry for every set, with one common cpt, overrides the defaults
    std::vector<TuneEntry> tuned(nsets);
    bool tuned_ok = getenv("EQS_TUNE_CACHE") != nullptr && env_int("EQS_CPT", 0) == 0 && env_int("EQS_KC", 0) == 0;
    int tuned_cpt = 0;
    if (tuned_ok) {
        const std::string arch = arch_name(c->device);
        for (int s = 0; s < nsets && tuned_ok; ++s) {
            tuned_ok = cache_lookup(getenv("EQS_TUNE_CACHE"), arch, grids[s], precision, &tuned[s]);
            if (tuned_ok && s > 0 && tuned[s].cpt != tuned[0].cpt) tuned_ok = false;
        }
        for (int s = 1; s < nsets && tuned_ok; ++s) tuned_ok = tuned[s].fnt == tuned[0].fnt;
        if (tuned_ok) tuned_cpt = tuned[0].cpt;
        if (tuned_ok && march_lds_bytes(tuned_cpt, max_nx, 8) > kMaxLds) tuned_ok = false;
        if (tuned_ok && c->sync1 &&
            !(fused_shape_ok(tuned_cpt, max_nx, tuned[0].fnt) &&
              fused_lds_bytes(tuned_cpt, max_nx, 8, tuned[0].fnt) <= c->fused_lds_cap))
            tuned_ok = false;
        if (tuned_ok) {
            cpt = tuned_cpt;
            if (c->sync1) c->fnt = tuned[0].fnt;
        }
    }
    c->cpt = cpt;
    c->max_nx = max_nx;

    size_t bytes = 0;
    const bool f32 = precision != EQS_FP64;
    std::vector<size_t> base(nsets);
    for (int s = 0; s < nsets; ++s) {
        SetHost &h = c->sets[s];
        memset(&h, 0, sizeof(h));
        h.g = grids[s];
        h.plane = grids[s].nx * grids[s].ny;
        h.n = h.plane * grids[s].nz;
        choose_tiling(h, cpt, c->fnt);
        if (tuned_ok) set_tiling(h, tuned_cpt, tuned[s].kc, tuned[s].nflat, c->fnt, c->sync1 ? tuned[s].ford : 0);
        base[s] = bytes;
        bytes += set_ws_bytes(h, f32, max_partials(h));
    }
    c->ws_bytes = bytes;
    if (hipMalloc(&c->ws, bytes) != hipSuccess) { (void)hipGetLastError(); delete c; return EQS_ERR_NOMEM; }
    if (hipMalloc((void **)&c->d_desc, sizeof(SetDesc) * nsets) != hipSuccess ||
        hipMalloc((void **)&c->d_state, sizeof(SolveState) * nsets) != hipSuccess ||
        hipHostMalloc((void **)&c->h_desc, sizeof(SetDesc) * nsets, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_state, sizeof(SolveState) * nsets, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        eqsolve_destroy(c);
        return EQS_ERR_NOMEM;
    }
    memset(c->h_desc, 0, sizeof(SetDesc) * nsets);
    memset(c->h_state, 0, sizeof(SolveState) * nsets);
    char *w = (char *)c->ws;
    for (int s = 0; s < nsets; ++s) {
        SetHost &h = c->sets[s];
        carve_set(h, w + base[s], f32, max_partials(h));
        fill_desc(c, s);
    }
    // zero counters and states once (kernels leave every counter at zero)
    if (hipMemsetAsync(c->ws, 0, bytes, c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_state, 0, sizeof(SolveState) * nsets, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_desc, c->h_desc, sizeof(SetDesc) * nsets, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        eqsolve_destroy(c);
        return EQS_ERR_HIP;
    }
    *out = c;
    return EQS_OK;
}

int eqsolve_set_preconditioner(eqs_ctx *c, int32_t kind, const eqs_mg_params *prm) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (kind == EQS_PRECOND_JACOBI) {
        const bool was_mg = c->precond == EQS_PRECOND_MG;
        c->precond = EQS_PRECOND_JACOBI;
        if (!was_mg) return EQS_OK;
        retile_for_precond(c);
        clear_graphs(c);
        return upload_desc(c, 0, c->nsets);
    }
    if (kind != EQS_PRECOND_MG || c->precision != EQS_FP64) return EQS_ERR_ARG;
    MgParams p{0.8, 1.0, 30, 512};
    if (prm) p = MgParams{prm->omega, prm->gamma, prm->coarse_sweeps, prm->coarse_cells};
    if (!(p.omega > 0.0 && p.omega < 2.0) || !(p.gamma > 0.0 && p.gamma <= 4.0) || p.coarse_sweeps < 1 ||
        p.coarse_sweeps > 100000 || p.coarse_cells < 1 || p.coarse_cells > kMgCoarsestMax)
        return EQS_ERR_ARG;
    // levels: halve every dimension (rounding up) until at most coarse_cells cells remain
    std::vector<std::vector<MgLevel>> mg(c->nsets);
    size_t bytes = 0;
    for (int s = 0; s < c->nsets; ++s) {
        const eqs_grid &g = c->sets[s].g;
        MgLevel l0{};
        l0.nx = g.nx;
        l0.ny = g.ny;
        l0.nz = g.nz;
        l0.n = c->sets[s].n;
        mg[s].push_back(l0);
        bytes += 7 * align_up((size_t)l0.n * 4);   // level 0's FP32 coefficients
        while (mg[s].back().n > p.coarse_cells && mg[s].back().n > 1 && (int)mg[s].size() < kMgMaxLevels) {
            const MgLevel &f = mg[s].back();
            MgLevel q{};
            q.nx = (f.nx + 1) / 2;
            q.ny = (f.ny + 1) / 2;
            q.nz = (f.nz + 1) / 2;
            q.n = q.nx * q.ny * q.nz;
            mg[s].push_back(q);
            bytes += 9 * align_up((size_t)q.n * 8);
        }
        if (mg[s].back().n > kMgCoarsestMax) return EQS_ERR_ARG;
    }
    void *ws = nullptr;
    if (bytes && hipMalloc(&ws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return EQS_ERR_NOMEM;
    }
    if (!c->d_mg && hipMalloc((void **)&c->d_mg, sizeof(MgLevel) * kMgMaxLevels * c->nsets) != hipSuccess) {
        (void)hipGetLastError();
        if (ws) (void)hipFree(ws);
        return EQS_ERR_NOMEM;
    }
    char *q = (char *)ws;
    std::vector<MgLevel> table((size_t)kMgMaxLevels * c->nsets);
    for (int s = 0; s < c->nsets; ++s)
        for (size_t l = 0; l < mg[s].size(); ++l) {
            MgLevel &L = mg[s][l];
            if (l == 0) {
                for (int k = 0; k < 7; ++k) {
                    L.a32[k] = (float *)q;
                    q += align_up((size_t)L.n * 4);
                }
            } else {
                for (int k = 0; k < 7; ++k) {
                    L.a[k] = (double *)q;
                    q += align_up((size_t)L.n * 8);
                }
                L.r = (double *)q;
                q += align_up((size_t)L.n * 8);
                L.z = (double *)q;
                q += align_up((size_t)L.n * 8);
            }
            table[(size_t)s * kMgMaxLevels + l] = L;
        }
    if (hipMemcpyAsync(c->d_mg, table.data(), sizeof(MgLevel) * table.size(), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        if (ws) (void)hipFree(ws);
        c->broken = true;
        return EQS_ERR_HIP;
    }
    clear_graphs(c);
    if (c->mg_ws) (void)hipFree(c->mg_ws);
    c->mg_ws = ws;
    c->mg = std::move(mg);
    c->mgp = p;
    c->mgp.coarse_sym = env_int("EQS_MG_CSYM", 1) != 0 ? 1 : 0;
    c->precond = EQS_PRECOND_MG;
    retile_for_precond(c);
    clear_graphs(c);
    return upload_desc(c, 0, c->nsets);
}

int eqsolve_set_step_form(eqs_ctx *c, int32_t form) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if ((form != EQS_STEP_SCALED && form != EQS_STEP_UNSCALED) || c->precision != EQS_FP64) return EQS_ERR_ARG;
    if (form != c->step_form) {
        c->step_form = form;
        clear_graphs(c);
    }
    return EQS_OK;
}

int eqsolve_debug_precond(eqs_ctx *c, int32_t set, const double *const diag[7], const double *r, double *z,
                          int32_t *levels) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (c->precond != EQS_PRECOND_MG || set < 0 || set >= c->nsets || !diag_ok(diag) || !r || !z || r == z)
        return EQS_ERR_ARG;
    SetDesc &d = c->h_desc[set];
    for (int k = 0; k < 7; ++k) d.a[k] = diag[k];
    int rc = upload_desc(c, set, 1);
    if (rc) return rc;
    const Run R = make_run(c, set, 1, false);
    // through the set's own r and t buffers (the V-cycle takes its vectors from the set table)
    const size_t bytes = (size_t)c->sets[set].n * sizeof(double);
    if (hipMemcpyAsync(c->sets[set].r, r, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        mg_coarsen_all(c, set) != hipSuccess || mg_vcycle(R, 2, false, c->stream) != hipSuccess ||
        hipMemcpyAsync(z, c->sets[set].t, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        c->broken = true;
        return EQS_ERR_HIP;
    }
    if (levels) *levels = (int32_t)c->mg[set].size();
    return EQS_OK;
}

int eqsolve_destroy(eqs_ctx *c) {
    if (!c) return EQS_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    clear_graphs(c);
    if (c->mg_ws) (void)hipFree(c->mg_ws);
    if (c->d_mg) (void)hipFree(c->d_mg);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->ws) (void)hipFree(c->ws);
    if (c->d_desc) (void)hipFree(c->d_desc);
    if (c->d_state) (void)hipFree(c->d_state);
    if (c->h_desc) (void)hipHostFree(c->h_desc);
    if (c->h_state) (void)hipHostFree(c->h_state);
    (void)hipGetLastError();
    delete c;
    return EQS_OK;
}

int eqsolve_solve(eqs_ctx *c, int32_t set, const double *const diag[7], const double *b, double *x, double tol,
                  int32_t maxit, eqs_info *info) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (set < 0 || set >= c->nsets || !diag_ok(diag) || !b || !x) return EQS_ERR_ARG;
    if (!(tol > 0.0 && tol < 1.0) || maxit < 1) return EQS_ERR_ARG;
    if (aliases(x, diag, b)) return EQS_ERR_ARG;
    SetDesc &d = c->h_desc[set];
    for (int k = 0; k < 7; ++k) d.a[k] = diag[k];
    d.b = b;
    d.x = x;
    d.xf = nullptr;
    for (int k = 0; k < 7; ++k) d.g[k] = nullptr;
    d.mode = set_mode_for(c->precision);
    d.tol = tol;
    d.tol_inner = d.mode == MODE_FP32 ? tol : inner_tol();
    d.maxit = maxit;
    int rc = upload_desc(c, set, 1);
    if (rc) return rc;
    Run R = make_run(c, set, 1, false);
    rc = d.mode == MODE_FP64 ? run_fp64(R) : run_fp32(R);
    if (rc) return rc;
    if ((rc = R.readback())) return rc;
    write_info(c, set, info);
    return c->h_state[set].status;
}

int eqsolve_solve_batched(eqs_ctx *c, const double *const *const *diag, const double *const *b, double *const *x,
                          const double *tol, const int32_t *maxit, eqs_info *info) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (!diag || !b || !x || !tol || !maxit) return EQS_ERR_ARG;
    for (int s = 0; s < c->nsets; ++s) {
        if (!diag_ok(diag[s]) || !b[s] || !x[s]) return EQS_ERR_ARG;
        if (!(tol[s] > 0.0 && tol[s] < 1.0) || maxit[s] < 1) return EQS_ERR_ARG;
        if (aliases(x[s], diag[s], b[s])) return EQS_ERR_ARG;
    }
    for (int s = 0; s < c->nsets; ++s) {
        SetDesc &d = c->h_desc[s];
        for (int k = 0; k < 7; ++k) d.a[k] = diag[s][k];
        d.b = b[s];
        d.x = x[s];
        d.xf = nullptr;
        for (int k = 0; k < 7; ++k) d.g[k] = nullptr;
        d.mode = set_mode_for(c->precision);
        d.tol = tol[s];
        d.tol_inner = d.mode == MODE_FP32 ? tol[s] : inner_tol();
        d.maxit = maxit[s];
    }
    int rc = upload_desc(c, 0, c->nsets);
    if (rc) return rc;
    Run R = make_run(c, 0, c->nsets, false);
    rc = c->precision == EQS_FP64 ? run_fp64(R) : run_fp32(R);
    if (rc) return rc;
    if ((rc = R.readback())) return rc;
    int worst = EQS_OK;
    for (int s = 0; s < c->nsets; ++s) {
        if (info) write_info(c, s, info + s);
        worst = std::max(worst, (int)c->h_state[s].status);
    }
    for (int s = 0; s < c->nsets; ++s)
        if (c->h_state[s].status < 0) return c->h_state[s].status;
    return worst;
}

int eqsolve_adjoint(eqs_ctx *c, int32_t set, const double *const diag[7], const double *x, const double *w,
                    double *grad_b, double *const grad_diag[7], double tol, int32_t maxit, eqs_info *info) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (set < 0 || set >= c->nsets || !diag_ok(diag) || !x || !w || !grad_b) return EQS_ERR_ARG;
    if (!(tol > 0.0 && tol < 1.0) || maxit < 1) return EQS_ERR_ARG;
    if (aliases(grad_b, diag, w) || (const double *)grad_b == x) return EQS_ERR_ARG;
    SetDesc &d = c->h_desc[set];
    for (int k = 0; k < 7; ++k) d.a[k] = diag[k];
    d.b = w;
    d.x = grad_b;
    d.xf = x;
    for (int k = 0; k < 7; ++k) d.g[k] = grad_diag ? grad_diag[k] : nullptr;
    d.mode = MODE_ADJOINT;
    d.tol = tol;
    d.tol_inner = tol;
    d.maxit = maxit;
    int rc = upload_desc(c, set, 1);
    if (rc) return rc;
    if (c->precond == EQS_PRECOND_MG) {
        // A^T's rows into the set's scaled-coefficient buffers (unused by the multigrid iteration),
        // then the multigrid solve of A^T lambda = w on them: its hierarchy is built from A^T
        Run T = make_run(c, set, 1, false);
        if ((rc = T.L(K_TRANSPOSE))) return rc;
        // the set table is pinned host memory, read by the upload when it executes: the transpose
        // must have read this call's pointers before they are replaced
        EQS_HIP(hipStreamSynchronize(c->stream));
        for (int k = 1; k < 7; ++k) d.a[k] = c->sets[set].as[k - 1];
        if ((rc = upload_desc(c, set, 1))) return rc;
        Run R = make_run(c, set, 1, false);
        if ((rc = R.L(K_ZERO, nullptr, nullptr, 1))) return rc;  // lambda0 = 0
        if ((rc = run_fp64(R))) return rc;
        if ((rc = R.L(K_GRAD))) return rc;
        if ((rc = R.readback())) return rc;
        write_info(c, set, info);
        return c->h_state[set].status;
    }
    Run R = make_run(c, set, 1, true);
    if ((rc = R.L(K_ZERO, nullptr, nullptr, 1))) return rc;  // lambda0 = 0
    if ((rc = run_fp64(R))) return rc;
    if ((rc = R.L(K_GRAD))) return rc;
    if ((rc = R.readback())) return rc;
    write_info(c, set, info);
    return c->h_state[set].status;
}

int eqsolve_apply(eqs_ctx *c, int32_t set, const double *const diag[7], const double *x, double *y,
                  int32_t transpose) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (set < 0 || set >= c->nsets || !diag_ok(diag) || !x || !y || (const void *)x == (const void *)y)
        return EQS_ERR_ARG;
    SetDesc &d = c->h_desc[set];
    for (int k = 0; k < 7; ++k) d.a[k] = diag[k];
    int rc = upload_desc(c, set, 1);
    if (rc) return rc;
    Run R = make_run(c, set, 1, transpose != 0);
    if ((rc = R.L(K_APPLY, x, y))) return rc;
    EQS_HIP(hipStreamSynchronize(c->stream));
    return EQS_OK;
}

const char *eqsolve_strerror(int code) {
    switch (code) {
    case EQS_OK: return "converged";
    case EQS_NOT_CONVERGED: return "not converged (iteration limit, or refinement stopped reducing the residual)";
    case EQS_BREAKDOWN: return "BiCGSTAB breakdown";
    case EQS_NONFINITE: return "non-finite value in the input or an iterate";
    case EQS_ERR_ARG: return "invalid argument";
    case EQS_ERR_NOMEM: return "device allocation failed";
    case EQS_ERR_HIP: return "HIP runtime error";
    case EQS_ERR_STATE: return "context unusable";
    case EQS_ERR_SIZE: return "system exceeds the static workspace of eqsolve_solve_noalloc";
    default: return "unknown eqsolve code";
    }
}

// introspection used by tests and the benchmark (not part of the solver contract)
int eqsolve_debug_layout(const eqs_ctx *c, int32_t set, int32_t *out8) {  // 12 entries
    if (!c || set < 0 || set >= c->nsets || !out8) return EQS_ERR_ARG;
    const SetHost &h = c->sets[set];
    out8[0] = c->cpt;
    out8[1] = h.S;
    out8[2] = h.KC;
    out8[3] = h.NKC;
    out8[4] = h.ntiles;
    out8[5] = (int32_t)std::min<uint64_t>(c->readbacks, 0x7fffffff);
    out8[6] = c->sync1 ? 1 : 3;
    out8[7] = h.nflat;
    out8[8] = c->fnt;
    out8[9] = h.fS;
    out8[10] = h.fntiles;
    out8[11] = h.ford;
    return EQS_OK;
}

int eqsolve_autotune(eqs_ctx *c, const char *cache_path, int32_t iters) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (iters < 1) iters = 6;
    iters = std::min(iters, 64);
    const std::string arch = arch_name(c->device);
    size_t nmax = 0;
    for (int s = 0; s < c->nsets; ++s) nmax = std::max(nmax, (size_t)c->sets[s].n);
    double *tmp = nullptr;
    if (hipMalloc((void **)&tmp, 9 * nmax * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return EQS_ERR_NOMEM;
    }
    // a well-conditioned synthetic system of each set's shape: a_P = 7, a_nb = 1, b = 1
    int rc = EQS_OK;
    for (int k = 0; k < 9 && rc == EQS_OK; ++k)
        if (launch_fill(tmp + k * nmax, (long)nmax, k == 0 ? 7.0 : 1.0, c->stream) != hipSuccess) rc = EQS_ERR_HIP;
    const int kcs[] = {1, 2, 4, 8, 16, 32, 48, 64};
    const int flats[] = {256, 512, 1024, 2048, 4096};
    const int old_cpt = c->cpt, old_fnt = c->fnt;
    double best_total = 1e300;
    int best_cpt = old_cpt, best_fnt = old_fnt;
    std::vector<TuneEntry> best(c->nsets), cur(c->nsets);
    // cells per thread and, for the single-sync step, its block size (256 or 512 threads), which
    // every set of the context shares; per set the planes per chunk and the tile order
    for (int cpt = 1; cpt <= 2 && rc == EQS_OK; ++cpt) {
        if (march_lds_bytes(cpt, c->max_nx, 8) > kMaxLds) continue;
        for (int fnt : {256, 512}) {
            if (rc != EQS_OK) break;
            if (!c->sync1 && fnt != 256) continue;
            if (c->sync1 && !(fused_shape_ok(cpt, c->max_nx, fnt) &&
                              fused_lds_bytes(cpt, c->max_nx, 8, fnt) <= c->fused_lds_cap))
                continue;
            c->cpt = cpt;
            c->fnt = fnt;
            clear_graphs(c);
            double total = 0.0;
            for (int s = 0; s < c->nsets && rc == EQS_OK; ++s) {
                SetHost &h = c->sets[s];
                const int kc0 = h.KC;
                TuneEntry b{cpt, kc0, h.nflat, fnt, 0, 1e300};
                for (int kc : kcs) {
                    if (kc > h.g.nz && kc != kcs[0]) continue;
                    for (int ford = 0; ford <= (c->sync1 ? 1 : 0); ++ford) {
                        set_tiling(h, cpt, kc, h.nflat, fnt, ford);
                        const double us = time_steps(c, s, 1, tmp, nmax, iters);
                        if (us == -1.0) { rc = EQS_ERR_HIP; break; }
                        if (us > 0 && us < b.us) b = TuneEntry{cpt, kc, h.nflat, fnt, ford, us};
                    }
                    if (rc != EQS_OK) break;
                }
                if (rc != EQS_OK) break;
                // a set too small to iterate this long keeps its default depth
                if (b.us >= 1e300) b = TuneEntry{cpt, kc0, h.nflat, fnt, 0, 0.0};
                cur[s] = b;
                total += b.us;
            }
            if (rc == EQS_OK && total < best_total) {
                best_total = total;
                best_cpt = cpt;
                best_fnt = fnt;
                best = cur;
            }
        }
    }
    // pointwise block count, with the chosen march tiling.  The single-sync step launches no
    // pointwise kernel, so timing it cannot choose one: those contexts keep the default count
    // (measured on the 128x256x128 pressure-like system, whose multigrid iteration runs pointwise
    // passes every step: 8.53-8.54 ms per solve with 512 or 1024 blocks, 8.62 with 2048, 8.93 with
    // 4096, 8.82 with 256)
    c->cpt = best_cpt;
    c->fnt = best_fnt;
    clear_graphs(c);
    for (int s = 0; s < c->nsets && rc == EQS_OK && !c->sync1; ++s) {
        SetHost &h = c->sets[s];
        for (int nf : flats) {
            set_tiling(h, best_cpt, best[s].kc, nf, best_fnt, best[s].ford);
            if (h.nflat != nf) continue;
            const double us = time_steps(c, s, 1, tmp, nmax, iters);
            if (us == -1.0) { rc = EQS_ERR_HIP; break; }
            if (us > 0 && us < best[s].us) best[s] = TuneEntry{best_cpt, best[s].kc, nf, best_fnt, best[s].ford, us};
        }
    }
    // Several sets: their batched launch holds every set's tiles at once, so the depths that are
    // fastest for each set alone can leave the last round of blocks part-empty.  Time the batched
    // step under the per-set choice and under one common depth for all sets, and keep the fastest
    // (for this context only: the cache keeps the per-set choice, which a context of one set wants).
    // A batched launch holds every set's tiles at once, so it is also timed under one common
    // depth for all sets, in either tile order, with either block size of the single-sync step
    // (the batch fills the device where one set's launch leaves its last round part-empty); the
    // fastest wins for this context (the cache keeps the per-set choice, which a context of one
    // set wants).
    std::vector<TuneEntry> chosen = best;
    int chosen_fnt = best_fnt;
    if (rc == EQS_OK && c->nsets > 1 && c->sync1) {
        c->fnt = best_fnt;
        for (int s = 0; s < c->nsets; ++s)
            set_tiling(c->sets[s], best_cpt, best[s].kc, best[s].nflat, best_fnt, best[s].ford);
        clear_graphs(c);
        double best_us = time_steps(c, 0, c->nsets, tmp, nmax, iters);
        if (best_us == -1.0) rc = EQS_ERR_HIP;
        const int common[] = {8, 12, 16, 24, 32, 48, 64, 96};
        for (int fnt : {256, 512}) {
            if (!(fused_shape_ok(best_cpt, c->max_nx, fnt) &&
                  fused_lds_bytes(best_cpt, c->max_nx, 8, fnt) <= c->fused_lds_cap))
                continue;
            c->fnt = fnt;
            for (int ford = 0; ford <= 1; ++ford)
                for (int kc : common) {
                    if (rc != EQS_OK || best_us <= 0) break;
                    for (int s = 0; s < c->nsets; ++s)
                        set_tiling(c->sets[s], best_cpt, kc, best[s].nflat, fnt, ford);
                    clear_graphs(c);
                    const double us = time_steps(c, 0, c->nsets, tmp, nmax, iters);
                    if (us == -1.0) { rc = EQS_ERR_HIP; break; }
                    if (us > 0 && us < 0.98 * best_us) {
                        best_us = us;
                        chosen_fnt = fnt;
                        for (int s = 0; s < c->nsets; ++s)
                            chosen[s] = TuneEntry{best_cpt, c->sets[s].KC, best[s].nflat, fnt, ford, us};
                    }
                }
        }
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    (void)hipGetLastError();
    if (rc != EQS_OK) {
        c->broken = true;
        return rc;
    }
    if ((rc = apply_tuning(c, best_cpt, chosen_fnt, chosen))) return rc;
    const char *path = cache_path ? cache_path : getenv("EQS_TUNE_CACHE");
    for (int s = 0; s < c->nsets; ++s) cache_store(path, arch, c->sets[s].g, c->precision, best[s]);
    return EQS_OK;
}

int eqsolve_debug_profile(eqs_ctx *c, int32_t kind_mask, int32_t every) {
    if (!c || c->broken) return EQS_ERR_STATE;
    if (every < 1) return EQS_ERR_ARG;
    c->profile_mask = (uint32_t)kind_mask;
    c->profile_every = every;
    for (int i = 0; i < 32; ++i) {
        c->kcount[i] = 0;
        c->kms[i] = 0.0;
        c->kseen[i] = 0;
    }
    return EQS_OK;
}

int eqsolve_debug_kernel_stats(const eqs_ctx *c, int32_t kind, int32_t fp32, int64_t *count, double *total_ms) {
    if (!c || kind < 0 || kind >= 32 || !count || !total_ms) return EQS_ERR_ARG;
    const int i = kind * 2 + (fp32 ? 1 : 0);
    *count = c->kcount[i];
    *total_ms = c->kms[i];
    return EQS_OK;
}

}  // extern "C"
