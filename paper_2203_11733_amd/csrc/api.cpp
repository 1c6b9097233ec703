// C ABI of libgbem: contexts, the extraction pipeline, the serving loop and
// the stage entry points.  Every numerical step runs in the HIP kernels of
// this library; the host code only sequences launches, sizes workspaces and
// moves the (small) inputs and outputs.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <memory>
#include <thread>
#include <vector>

#include "admission.h"
#include "gbem_internal.h"

namespace gbem {

static thread_local std::string t_err;
void set_error(const std::string &msg) { t_err = msg; }

// Gauss-Legendre rule: Newton iteration on P_p (Bonnet recurrence, long
// double) from Tricomi's asymptotic node estimates.
void gauss_legendre(int p, double *xo, double *wo)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 1; i <= p; ++i) {
        long double th = pi * (4.0L * i - 1.0L) / (4.0L * p + 2.0L);
        long double x = (1.0L - 1.0L / (8.0L * p * p) + 1.0L / (8.0L * p * p * p)) * cosl(th);
        long double dp = 1.0L;
        for (int it = 0; it < 50; ++it) {
            long double p0 = 1.0L, p1 = x;
            for (int k = 2; k <= p; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (p == 1) p0 = 1.0L;
            dp = p * (p0 - x * p1) / (1.0L - x * x);
            long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        // nodes ascending: i = 1 is the largest root
        const int idx = p - i;
        xo[idx] = (double)x;
        wo[idx] = (double)(1.0L / ((1.0L - x * x) * dp * dp));   // = w/2 (halved weight)
    }
}

void gauss_legendre_rule(int p, GaussRule *r)
{
    memset(r, 0, sizeof(*r));
    gauss_legendre(p, r->x, r->w);
    for (int a = 0; a < p; ++a) {
        r->xf[a] = (float)r->x[a];
        for (int b = 0; b < p; ++b) {
            r->ww[a * p + b] = r->w[a] * r->w[b];
            r->wwf[a * p + b] = (float)r->ww[a * p + b];
        }
    }
}

// ------------------------------------------------------------------------
// device buffers
// ------------------------------------------------------------------------
// A bump allocator over a fixed device region (the no-allocation entry
// point's scratch array): buffers are carved in call order and the whole
// region is handed back at once (reset) before the next call.
struct Arena {
    unsigned char *base = nullptr;
    size_t size = 0, used = 0;
    bool exhausted = false;   // a request did not fit (the call fails with GBEM_ENOMEM)
    void reset()
    {
        used = 0;
        exhausted = false;
    }
};

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    Arena *arena = nullptr;   // set: memory comes from the arena, never from hipMalloc
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (arena) {
            const size_t want = (bytes + 255) & ~(size_t)255;
            if (want > arena->size - arena->used) {
                arena->exhausted = true;
                return hipErrorOutOfMemory;
            }
            p = arena->base + arena->used;
            arena->used += want;
            cap = want;
            return hipSuccess;
        }
        release();
        size_t want = (bytes + 4095) & ~(size_t)4095;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
    void release()
    {
        if (p && !arena) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Small results the host reads during an extraction, in pinned memory so a
// read is one DMA (no staging copy), gathered so that each host wait covers
// all of them.
constexpr double kEps0 = 8.8541878128e-12;   // vacuum permittivity, F/m

struct Readback {
    int64_t nnz;
    int32_t bad, info, perr, serr;   // info, perr: flags[1], flags[2] (pivot status, panel wait error)
    double bn[kMaxRhs], rn[kMaxRhs];
    double C[kMaxRhs * kMaxRhs];
};

struct Workspace {
    DevBuf lo, hi, cond, pan, cnt, rowptr, nrow, ncol, A, F, Winv, Pw, P16, B, X, R, s, partial, C,
        flags, norms, sflags, rpart, semi, nmask;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t evrb = nullptr;          // readback point
    Readback *rb = nullptr;             // pinned host memory
    bool events_ok = false;
    SolveSync sync;
    Prof prof;
    hipStream_t side = nullptr;         // look-ahead stream of the factorisation
    // the factorisation's look-ahead runs on the pipeline's own stream (same
    // results, no overlap inside the job): for serving workers that share the
    // GPU with other jobs, whose kernels fill the gaps instead, and for the
    // no-allocation entry, which keeps no stream of its own
    bool lookahead_on_main = false;
    std::vector<hipEvent_t> fev;        // its event pool

    hipError_t ensure_side()
    {
        if (side) return hipSuccess;
        return hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    }

    // flags of the persistent solves: zeroed once when (re)allocated; the
    // epoch restarts with them
    // (published words are epoch-tagged: zero tags never match an epoch >= 1)
    // layout: flag words (error, tickets, per-block flags), published blocks, M_k, N_k, M2_k, N2_k
    static size_t sync_flag_bytes(int64_t npad) { return (((size_t)2 * (npad / kNB) * 4 + 256) + 255) / 256 * 256; }
    static size_t sync_bytes(int64_t npad)
    {
        return sync_flag_bytes(npad) + (size_t)2 * npad * kMaxPub * 8 + (size_t)4 * npad * kNB * 4;
    }
    hipError_t ensure_sync(int64_t npad, hipStream_t st)
    {
        const size_t nflag = sync_flag_bytes(npad);
        const size_t npub = (size_t)2 * npad * kMaxPub * 8;
        const size_t need = sync_bytes(npad);
        if (sflags.cap < need || sync_npad != npad) {
            hipError_t e = sflags.ensure(need);
            if (e != hipSuccess) return e;
            e = hipMemsetAsync(sflags.p, 0, need, st);
            if (e != hipSuccess) return e;
            sync.epoch = 0;
            sync.base_f = sync.base_b = 0;
            sync_npad = npad;
        }
        int32_t *f = sflags.as<int32_t>();
        sync.err = f;                      // word 0: error flag, words 1, 2: ticket counters
        sync.flags_f = f + 64;
        sync.flags_b = f + 64 + (nflag / 4 - 64) / 2;
        sync.pub = reinterpret_cast<uint64_t *>(sflags.as<char>() + nflag);
        sync.sub = reinterpret_cast<float *>(sflags.as<char>() + nflag + npub);
        return hipSuccess;
    }
    int64_t sync_npad = -1;

    static constexpr int kBuffers = 25;
    template <typename Fn> void each(Fn f)
    {
        DevBuf *all[kBuffers] = {&lo, &hi, &cond, &pan, &cnt, &rowptr, &nrow, &ncol, &A, &F, &Winv, &Pw,
                                 &P16, &B, &X, &R, &s, &partial, &C, &flags, &norms, &sflags, &rpart, &semi, &nmask};
        for (auto *b : all) f(*b);
    }
    size_t bytes()
    {
        size_t t = 0;
        each([&](DevBuf &b) { t += b.cap; });
        return t;
    }
    void release_all()
    {
        each([](DevBuf &b) { b.release(); });
    }
    hipError_t init_events()
    {
        if (events_ok) return hipSuccess;
        for (auto &e : ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        hipError_t r = hipEventCreateWithFlags(&evrb, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        void *h = nullptr;
        if ((r = hipHostMalloc(&h, sizeof(Readback), hipHostMallocDefault)) != hipSuccess) return r;
        rb = static_cast<Readback *>(h);
        events_ok = true;
        return hipSuccess;
    }
    // executables of captured launch sequences (opts.graph), keyed by order,
    // factor dtype and right-hand sides; a new capture is applied to the
    // matching one with hipGraphExecUpdate (instantiated when the topology
    // differs or none matches)
    // The key also holds the addresses of the buffers the captured copies
    // read or write (flags, B, X, norms, solve flags): an update then only
    // changes kernel arguments, and a reallocated buffer means a new
    // executable.
    static constexpr int kCopyBufs = 5;
    struct GraphExec {
        int64_t npad;
        int dtype, m;
        const void *bufs[kCopyBufs];
        hipGraphExec_t exec;
    };
    std::vector<GraphExec> gexec;
    static constexpr size_t kMaxGraphs = 8;
    hipError_t launch_graph(hipGraph_t g, int64_t npad, int dtype, int m, hipStream_t st, bool &instantiated)
    {
        instantiated = false;
        const void *bufs[kCopyBufs] = {flags.p, B.p, X.p, norms.p, sflags.p};
        GraphExec *slot = nullptr;
        for (auto &x : gexec)
            if (x.npad == npad && x.dtype == dtype && x.m == m && std::equal(bufs, bufs + kCopyBufs, x.bufs))
                slot = &x;
        hipError_t e = hipSuccess;
        if (slot) {
            hipGraphNode_t bad_node = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            e = hipGraphExecUpdate(slot->exec, g, &bad_node, &res);
            if (e != hipSuccess || res != hipGraphExecUpdateSuccess) {
                (void)hipGetLastError();   // a topology mismatch is not an error here
                (void)hipGraphExecDestroy(slot->exec);
                slot->exec = nullptr;
                if ((e = hipGraphInstantiate(&slot->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
                    gexec.erase(gexec.begin() + (slot - gexec.data()));
                    return e;
                }
                instantiated = true;
            }
        } else {
            if (gexec.size() >= kMaxGraphs) {
                (void)hipGraphExecDestroy(gexec.front().exec);
                gexec.erase(gexec.begin());
            }
            GraphExec x{npad, dtype, m, {}, nullptr};
            std::copy(bufs, bufs + kCopyBufs, x.bufs);
            if ((e = hipGraphInstantiate(&x.exec, g, nullptr, nullptr, 0)) != hipSuccess) return e;
            gexec.push_back(x);
            slot = &gexec.back();
            instantiated = true;
        }
        return hipGraphLaunch(slot->exec, st);
    }

    // buffers of the multi-dielectric entries (kept between calls like the
    // rest of the context's workspace)
    struct DlBufs {
        DevBuf tab, epsb, Q, M, Mt, B, Bn, Z, N, X, R, D, C, nrm, part, qrow, qcol;
        void release()
        {
            for (DevBuf *b : {&tab, &epsb, &Q, &M, &Mt, &B, &Bn, &Z, &N, &X, &R, &D, &C, &nrm, &part, &qrow, &qcol})
                b->release();
        }
    } dl;

    ~Workspace()
    {
        for (auto &x : gexec) (void)hipGraphExecDestroy(x.exec);
        dl.release();
        release_all();
        if (events_ok) {
            for (auto &e : ev) (void)hipEventDestroy(e);
            (void)hipEventDestroy(evrb);
            (void)hipHostFree(rb);
        }
        for (auto &e : fev) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }
};

// Device bytes one extraction holds at most: the buffers run_pipeline sizes,
// from the same helpers, for the requested factor and every fallback level
// above it (a failed or stalled 16-bit factor retries in FP32, then FP64).
// The near list is estimated at 512 pairs per row (at most n(n+1)/2); the
// real size is only known after the near test.
static size_t chunks_of(int64_t n) { return (size_t)((n + 1023) / 1024); }
static size_t page_round(size_t b) { return b ? (b + 4095) & ~(size_t)4095 : 0; }   // DevBuf::ensure's unit

// Bytes of each workspace buffer a job may allocate (Workspace::each order),
// for the requested factor and every fallback level above it (a failed or
// stalled 16-bit factor retries in FP32, then FP64).  The near list is
// estimated at 512 pairs per row (at most n(n+1)/2); its real size is only
// known after the near test.  include_near/include_mesh: the near list and
// the device copy of the mesh and C (what a synchronous call brings in).
static std::array<size_t, Workspace::kBuffers> buffer_needs(int64_t n, int m, int factor_dtype, bool include_near,
                                                            bool include_mesh)
{
    const int64_t npad = round_up(n, kPad);
    const int64_t nnz = std::min<int64_t>(n * 512, n * (n + 1) / 2);
    const bool low = factor_dtype != GBEM_F64;
    size_t w = 0, q = 64;
    for (int d = factor_dtype;; d = d == GBEM_F32 ? GBEM_F64 : GBEM_F32) {
        w = std::max(w, chol_winv_bytes(d, npad));
        q = std::max(q, chol_panel16_bytes(d, npad));
        if (d == GBEM_F64) break;
    }
    const size_t mesh3 = include_mesh ? (size_t)n * 3 * sizeof(double) : 0;
    const size_t near4 = include_near ? sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1) : 0;
    // lo, hi, cond, pan, cnt, rowptr, nrow, ncol, A, F, Winv, Pw, P16, B, X, R, s, partial, C, flags,
    // norms, sflags, rpart, semi, nmask
    const size_t v[Workspace::kBuffers] = {
        mesh3, mesh3, include_mesh ? (size_t)n * sizeof(int32_t) : 0,
        sizeof(Panel) * (size_t)n, sizeof(int64_t) * (size_t)n, sizeof(int64_t) * (size_t)(n + 1),
        near4, near4,
        (size_t)npad * npad * 8, low ? (size_t)npad * npad * 4 : 0, w, chol_panel_bytes(factor_dtype, npad), q,
        (size_t)npad * m * 8, (size_t)npad * m * 8, low ? (size_t)npad * m * 8 : 0, low ? (size_t)npad * 8 : 0,
        chunks_of(n) * m * m * 8, include_mesh ? sizeof(double) * m * m : 0, 64,
        sizeof(double) * 2 * kMaxRhs, Workspace::sync_bytes(npad),
        low ? (size_t)residual_splits((int)npad) * m * npad * 8 : 0, include_near ? near_semi_bytes(nnz) : 0,
        sizeof(uint64_t) * (size_t)n * near_mask_words(n)};
    std::array<size_t, Workspace::kBuffers> out;
    for (int i = 0; i < Workspace::kBuffers; ++i) out[i] = page_round(v[i]);
    return out;
}
// Device bytes one extraction holds at most in an empty workspace.
static size_t footprint(int64_t n, int m, int factor_dtype)
{
    size_t t = 0;
    for (size_t b : buffer_needs(n, m, factor_dtype, true, true)) t += b;
    return t;
}
// Bytes the workspace holds after a job with these needs: every buffer
// ends at the larger of its current capacity and the job's need.
static size_t grown_bytes(Workspace &ws, const std::array<size_t, Workspace::kBuffers> &need)
{
    size_t t = 0;
    int i = 0;
    ws.each([&](DevBuf &b) { t += std::max(b.cap, need[i++]); });
    return t;
}

static gbem_status dev_fail(hipError_t e, const char *where)
{
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? GBEM_ENOMEM : GBEM_EDEVICE;
}

#define HIPCHK(call, where)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return dev_fail(e_, where);     \
    } while (0)

static bool opts_ok(const gbem_opts &o, std::string &why)
{
    if (o.far_order < 1 || o.far_order > kMaxOrder || o.far_order == 7) {
        why = "far_order must be 1..6 or 8";
        return false;
    }
    // the near test is strict (dist^2 < eta^2 diam^2): with eta = 0 not even a
    // panel and itself would be near, and the far rule would put r = 0 into
    // 1/r on the self pairs
    if (!(o.near_eta >= kMinNearEta) || !isfinite(o.near_eta)) {
        why = "near_eta must be a finite number >= 1e-6 (pairs at zero separation, a panel with itself "
              "included, must be near)";
        return false;
    }
    if (o.far_dtype != GBEM_F64 && o.far_dtype != GBEM_F32) {
        why = "far_dtype must be GBEM_F64 or GBEM_F32";
        return false;
    }
    if (o.factor_dtype < GBEM_F64 || o.factor_dtype > GBEM_BF16) {
        why = "unknown factor_dtype";
        return false;
    }
    if (o.factor_dtype != GBEM_F64 && (!(o.refine_tol > 0.0) || o.max_refine < 0)) {
        why = "refinement needs refine_tol > 0 and max_refine >= 0";
        return false;
    }
    if (o.graph != 0 && o.graph != 1) {
        why = "graph must be 0 or 1";
        return false;
    }
    return true;
}

static bool mesh_header_ok(const gbem_mesh *m, std::string &why)
{
    if (!m || m->n_panels <= 0 || !m->lo || !m->hi || !m->conductor) {
        why = "mesh needs n_panels > 0 and lo/hi/conductor arrays";
        return false;
    }
    if (m->n_conductors < 1 || m->n_conductors > kMaxRhs) {
        why = "n_conductors must be in 1..64";
        return false;
    }
    if (!(m->eps_r > 0.0) || !(m->length_unit_m > 0.0) || !isfinite(m->eps_r) || !isfinite(m->length_unit_m)) {
        why = "eps_r and length_unit_m must be positive and finite";
        return false;
    }
    if (m->basis != GBEM_BASIS_P0) {
        why = "basis must be GBEM_BASIS_P0 (piecewise constant, the only basis of the method)";
        return false;
    }
    return true;
}

struct Timing {
    float assemble = 0, factor = 0, solve = 0, total = 0;
};

// kAssembled: A only; kScaled: A and the FP32 factor input F (low-precision
// factor); kFull: the whole extraction
enum class Stop { kAssembled, kScaled, kFull };

// The extraction pipeline on one stream and workspace.  Mesh arrays and C
// are device pointers.
// hC (optional): host copy of C, fetched with the final wait.
static gbem_status run_pipeline(Workspace &ws, hipStream_t st, int n, int m, const double *dlo,
                                const double *dhi, const int32_t *dcond, double eps_r, double lu,
                                const gbem_opts &o, double *dC, gbem_report *rep, Stop stop,
                                double *hC = nullptr)
{
    const int64_t npad = round_up(n, kPad);
    HIPCHK(ws.init_events(), "hipEventCreate");
    HIPCHK(ws.pan.ensure(sizeof(Panel) * n), "alloc panels");
    HIPCHK(ws.cnt.ensure(sizeof(int64_t) * n), "alloc near counts");
    HIPCHK(ws.rowptr.ensure(sizeof(int64_t) * (n + 1)), "alloc row_ptr");
    HIPCHK(ws.nmask.ensure(sizeof(uint64_t) * (size_t)n * near_mask_words(n)), "alloc near masks");
    HIPCHK(ws.flags.ensure(64), "alloc flags");
    HIPCHK(ws.A.ensure((size_t)npad * npad * 8), "alloc A");
    HIPCHK(ws.B.ensure((size_t)npad * m * 8), "alloc B");
    HIPCHK(ws.norms.ensure(sizeof(double) * 2 * kMaxRhs), "alloc norms");
    int32_t *flags = ws.flags.as<int32_t>();   // [0] bad panel, [1] factor info
    double *A = ws.A.as<double>();
    const int64_t lda = npad;

    Prof &pf = ws.prof;
    pf.on = o.profile != 0;
    pf.mask = (uint32_t)o.profile;
    pf.reset();
    if (rep) {
        for (int c = 0; c < GBEM_K_COUNT; ++c) {
            rep->prof_ms[c] = rep->prof_flops[c] = rep->prof_bytes[c] = 0.0;
            rep->prof_launches[c] = 0;
        }
    }
    // opts.graph: the launches from the near-list fill to the first host wait
    // after it are captured into a graph (no host waits, allocations, memset
    // nodes or timing events inside; the guard ends a capture left open by an
    // error return)
    const bool use_graph = o.graph == 1 && stop == Stop::kFull && !pf.on;
    struct CaptureGuard {
        hipStream_t st;
        bool on = false;
        ~CaptureGuard()
        {
            if (!on) return;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
        }
    } cap{st};
    bool graph_used = false, graph_inst = false;
    const int dtype0 = o.factor_dtype;
    auto end_segment = [&]() -> hipError_t {
        if (!cap.on) return hipSuccess;
        cap.on = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (e != hipSuccess) return e;
        e = ws.launch_graph(g, npad, dtype0, m, st, graph_inst);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return e;
        graph_used = true;
        return hipEventRecord(ws.ev[2], st);   // the graph ends the "factor" stage
    };
    HIPCHK(hipEventRecord(ws.ev[0], st), "hipEventRecord");
    HIPCHK(hipMemsetAsync(flags, 0, 64, st), "hipMemsetAsync");
    int tok = pf.start(st, GBEM_K_OTHER);
    HIPCHK(launch_build_panels(dlo, dhi, dcond, n, m, ws.pan.as<Panel>(), flags, st), "build_panels");
    pf.stop(tok, GBEM_K_OTHER, 0.0, (double)n * (48 + 4 + 64), st);
    const double eta2 = o.near_eta * o.near_eta;
    const int tok_near = pf.start(st, GBEM_K_NEAR_LIST);
    HIPCHK(launch_near_count(dlo, dhi, n, eta2, ws.cnt.as<int64_t>(), ws.nmask.as<uint64_t>(), st), "near_count");
    HIPCHK(launch_exclusive_scan(ws.cnt.as<int64_t>(), n, ws.rowptr.as<int64_t>(), st), "scan");
    pf.stop(tok_near, GBEM_K_NEAR_LIST, 0.0, (double)n * (48 + 8 + 8), st, 2);
    double *B = ws.B.as<double>();
    HIPCHK(launch_rhs(dcond, n, (int)npad, m, B, npad, st), "rhs");
    double *bnorm = ws.norms.as<double>() + kMaxRhs;
    HIPCHK(launch_col_norms(B, npad, (int)npad, m, bnorm, st), "col_norms");

    // one host wait: near-list size, validation flag, panels per conductor;
    // the far field (which needs none of them) is queued first and runs
    // while the host waits
    Readback *rbk = ws.rb;
    HIPCHK(hipMemcpyAsync(&rbk->nnz, ws.rowptr.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st), "D2H nnz");
    HIPCHK(hipMemcpyAsync(&rbk->bad, flags, 4, hipMemcpyDeviceToHost, st), "D2H flag");
    HIPCHK(hipMemcpyAsync(rbk->bn, bnorm, sizeof(double) * m, hipMemcpyDeviceToHost, st), "D2H norms");
    HIPCHK(hipEventRecord(ws.evrb, st), "hipEventRecord");
    GaussRule rule;
    gauss_legendre_rule(o.far_order, &rule);
    // a low-precision factor works on F = S A S in FP32 (S = diag(A)^(-1/2)):
    // S comes from the panels' self integrals up front, and the far and near
    // passes write F beside A, so no pass over the finished A is needed
    float *Fasm = nullptr;
    const double *sasm = nullptr;
    if (stop != Stop::kAssembled && o.factor_dtype != GBEM_F64) {
        HIPCHK(ws.F.ensure((size_t)npad * npad * 4), "alloc F");
        HIPCHK(ws.s.ensure((size_t)npad * 8), "alloc s");
        HIPCHK(launch_self_scale(dlo, dhi, ws.pan.as<Panel>(), n, (int)npad, ws.s.as<double>(), st), "self scale");
        Fasm = ws.F.as<float>();
        sasm = ws.s.as<double>();
    }
    tok = pf.start(st, GBEM_K_FAR);
    HIPCHK(launch_far(ws.pan.as<Panel>(), n, (int)npad, o.far_order, rule, o.far_dtype, A, lda, st, Fasm, npad, sasm),
           "far");
    {
        const double p2 = (double)o.far_order * o.far_order;
        // 11 flops per evaluation of w_a w_b / |x_a - y_b|: 3 differences, 5 for the
        // squared norm, 1 reciprocal square root, 2 for the weighted sum
        pf.stop(tok, GBEM_K_FAR, 11.0 * p2 * p2 * (double)n * (n + 1) / 2.0,
                (double)npad * npad * 8.0 + (double)n * sizeof(Panel), st);
    }
    HIPCHK(hipEventSynchronize(ws.evrb), "hipEventSynchronize");
    const int64_t nnz = rbk->nnz;
    const int32_t bad = rbk->bad;
    double bn[kMaxRhs];
    for (int k = 0; k < m; ++k) bn[k] = rbk->bn[k];
    if (bad) {
        HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");   // the far kernel is done with the panels
        set_error("panel " + std::to_string(bad - 1) +
                  " is not an axis-aligned rectangle with exactly one zero extent, or its conductor id is out of range");
        return GBEM_EINVAL;
    }
    for (int k = 0; k < m; ++k)
        if (bn[k] == 0.0) {
            HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
            set_error("conductor " + std::to_string(k) + " has no panels");
            return GBEM_EINVAL;
        }

    HIPCHK(ws.nrow.ensure(sizeof(int32_t) * std::max<int64_t>(nnz, 1)), "alloc near rows");
    HIPCHK(ws.ncol.ensure(sizeof(int32_t) * std::max<int64_t>(nnz, 1)), "alloc near cols");
    HIPCHK(ws.semi.ensure(near_semi_bytes(nnz)), "alloc near queue");
    if (use_graph) {
        // everything the captured launches use, allocated (and the solve flags
        // zeroed) before the capture
        HIPCHK(ws.X.ensure((size_t)npad * m * 8), "alloc X");
        HIPCHK(ws.ensure_sync(npad, st), "alloc solve flags");
        HIPCHK(ws.Winv.ensure(chol_winv_bytes(dtype0, npad)), "alloc W");
        HIPCHK(ws.Pw.ensure(chol_panel_bytes(dtype0, npad)), "alloc panel");
        HIPCHK(ws.P16.ensure(std::max<size_t>(chol_panel16_bytes(dtype0, npad), 64)), "alloc panel16");
        if (dtype0 != GBEM_F64) {
            HIPCHK(ws.R.ensure((size_t)npad * m * 8), "alloc R");
            HIPCHK(ws.rpart.ensure((size_t)residual_splits((int)npad) * m * npad * 8), "alloc residual partials");
        }
        HIPCHK(ws.partial.ensure((size_t)chunks_of(n) * m * m * 8), "alloc partials");
        if (!ws.lookahead_on_main) HIPCHK(ws.ensure_side(), "side stream");
        HIPCHK(near_eval_upload_rule(st), "near rule");
        HIPCHK(hipEventRecord(ws.ev[1], st), "hipEventRecord");
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
        cap.on = true;
    }
    tok = pf.start(st, GBEM_K_NEAR_LIST);
    HIPCHK(launch_near_fill(ws.nmask.as<uint64_t>(), n, ws.rowptr.as<int64_t>(), ws.nrow.as<int32_t>(),
                            ws.ncol.as<int32_t>(), st), "near_fill");
    pf.stop(tok, GBEM_K_NEAR_LIST, 0.0, (double)n * (n + 64) / 16.0 + (double)nnz * 8, st);
    tok = pf.start(st, GBEM_K_NEAR_EVAL);
    HIPCHK(launch_near_eval(dlo, dhi, ws.pan.as<Panel>(), ws.nrow.as<int32_t>(), ws.ncol.as<int32_t>(), nnz,
                            A, lda, ws.semi.as<int32_t>(), st, Fasm, npad, sasm, !cap.on), "near_eval");
    pf.stop(tok, GBEM_K_NEAR_EVAL, 0.0, (double)nnz * (2 * 8 + 2 * 4 + 2 * 48), st);
    if (!cap.on) HIPCHK(hipEventRecord(ws.ev[1], st), "hipEventRecord");
    if (rep) {
        rep->n_near = nnz;
        rep->n_panels = n;
    }
    if (stop != Stop::kFull) {
        HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
        pf.collect(rep);
        return GBEM_OK;
    }

    HIPCHK(ws.X.ensure((size_t)npad * m * 8), "alloc X");
    HIPCHK(ws.ensure_sync(npad, st), "alloc solve flags");
    HIPCHK(launch_fill_i32(ws.sync.err, 1, 0, st), "clear solve flag");
    double *X = ws.X.as<double>();
    int dtype = o.factor_dtype;
    bool f_ready = Fasm != nullptr;   // F = S A S written by the assembly (consumed by the first factor)
    int iters = 0;
    double resid = 0.0;
    for (;;) {   // fallback loop: a failed low-precision factor retries one level up
        const size_t es = dtype == GBEM_F64 ? 8 : 4;
        HIPCHK(ws.Winv.ensure(chol_winv_bytes(dtype, npad)), "alloc W");
        HIPCHK(ws.Pw.ensure(chol_panel_bytes(dtype, npad)), "alloc panel");
        HIPCHK(ws.P16.ensure(std::max<size_t>(chol_panel16_bytes(dtype, npad), 64)), "alloc panel16");
        HIPCHK(launch_fill_i32(flags + 1, 1, 0, st), "clear pivot flag");
        void *Fm = A;
        if (dtype != GBEM_F64) {
            if (!f_ready) {   // a retry: the failed factor overwrote F
                HIPCHK(ws.F.ensure((size_t)npad * npad * es), "alloc F");
                HIPCHK(ws.s.ensure((size_t)npad * 8), "alloc s");
                tok = pf.start(st, GBEM_K_OTHER);
                HIPCHK(launch_jacobi_scale(A, lda, (int)npad, ws.s.as<double>(), st), "jacobi");
                HIPCHK(launch_scale_convert(A, lda, ws.s.as<double>(), (int)npad, ws.F.as<float>(), npad, st),
                       "scale_convert");
                pf.stop(tok, GBEM_K_OTHER, 2.0 * (double)npad * npad / 2.0, (double)npad * npad / 2.0 * 12.0, st,
                        2);
            }
            f_ready = false;
            Fm = ws.F.p;
        }
        hipStream_t la = st;
        if (!ws.lookahead_on_main) {
            HIPCHK(ws.ensure_side(), "side stream");
            la = ws.side;
        }
        HIPCHK(chol_factor(dtype, npad, Fm, lda, ws.Winv.p, ws.Pw.p, ws.P16.p, flags + 1, st, la, ws.fev, &pf),
               "cholesky");
        // The pivot status is read with the next host wait; the solves are
        // queued behind it regardless (on a failed factor they are discarded:
        // their termination does not depend on the values).
        HIPCHK(hipMemcpyAsync(&rbk->info, flags + 1, 8, hipMemcpyDeviceToHost, st), "D2H info");
        HIPCHK(chol_solve_prep(dtype, npad, Fm, lda, ws.Winv.p, ws.sync, st), "solve prep");
        if (!cap.on && !graph_used) HIPCHK(hipEventRecord(ws.ev[2], st), "hipEventRecord");
        HIPCHK(hipMemcpyAsync(X, B, (size_t)npad * m * 8, hipMemcpyDeviceToDevice, st), "copy B");
        if (dtype == GBEM_F64) {
            HIPCHK(chol_solve(dtype, npad, A, lda, ws.Winv.p, m, X, npad, ws.sync, st, &pf), "solve");
            iters = 0;      // no refinement on an FP64 factor (also after an escalation)
            resid = 0.0;
            break;
        }
        // mixed precision: X = S F^{-1} S B, then FP64 refinement with A
        const double *sv = ws.s.as<double>();
        HIPCHK(launch_scale_rows(X, npad, sv, (int)npad, m, st), "scale");
        HIPCHK(chol_solve(dtype, npad, Fm, lda, ws.Winv.p, m, X, npad, ws.sync, st, &pf), "solve");
        HIPCHK(launch_scale_rows(X, npad, sv, (int)npad, m, st), "scale");
        HIPCHK(ws.R.ensure((size_t)npad * m * 8), "alloc R");
        HIPCHK(ws.rpart.ensure((size_t)residual_splits((int)npad) * m * npad * 8), "alloc residual partials");
        double *R = ws.R.as<double>();
        double *rnorm = ws.norms.as<double>();
        bool retry = false;
        double prev = INFINITY;
        for (iters = 0;; ++iters) {
            tok = pf.start(st, GBEM_K_RESIDUAL);
            HIPCHK(launch_residual(A, lda, (int)npad, X, npad, B, npad, m, R, npad, ws.rpart.as<double>(), st),
                   "residual");
            pf.stop(tok, GBEM_K_RESIDUAL, 2.0 * (double)npad * npad * m,
                    (double)npad * npad * 8.0 + 3.0 * (double)npad * m * 8.0, st, 2);
            HIPCHK(launch_col_norms(R, npad, (int)npad, m, rnorm, st), "col_norms");
            HIPCHK(hipMemcpyAsync(rbk->rn, rnorm, sizeof(double) * m, hipMemcpyDeviceToHost, st), "D2H norms");
            HIPCHK(hipMemcpyAsync(&rbk->serr, ws.sync.err, 4, hipMemcpyDeviceToHost, st), "D2H solve flag");
            HIPCHK(end_segment(), "graph");
            HIPCHK(hipEventRecord(ws.evrb, st), "hipEventRecord");
            HIPCHK(hipEventSynchronize(ws.evrb), "hipEventSynchronize");
            if (rbk->perr) {
                set_error("Cholesky: a panel wait exceeded its poll limit");
                return GBEM_EDEVICE;
            }
            if (iters == 0 && rbk->info != 0) {   // the low-precision factor failed
                retry = true;
                break;
            }
            const double *rn = rbk->rn;
            if (rbk->serr) {
                set_error("triangular solve: a block wait exceeded its poll limit");
                return GBEM_EDEVICE;
            }
            resid = 0.0;
            for (int k = 0; k < m; ++k) resid = std::max(resid, sqrt(rn[k] / bn[k]));
            if (resid <= o.refine_tol) break;
            // NaN or infinite, not contracting by at least half per sweep, or
            // out of sweeps: the factor is too weak for this matrix, and the
            // extraction retries one precision level up (as on a bad pivot)
            if (!isfinite(resid) || !(resid < 0.5 * prev) || iters >= o.max_refine) {
                retry = true;
                break;
            }
            prev = resid;
            HIPCHK(launch_scale_rows(R, npad, sv, (int)npad, m, st), "scale");
            HIPCHK(chol_solve(dtype, npad, Fm, lda, ws.Winv.p, m, R, npad, ws.sync, st, &pf), "solve");
            HIPCHK(launch_scale_rows(R, npad, sv, (int)npad, m, st), "scale");
            HIPCHK(launch_axpy_cols(X, npad, R, npad, (int)npad, m, st), "update");
        }
        if (retry) {
            dtype = (dtype == GBEM_F32) ? GBEM_F64 : GBEM_F32;   // BF16/F16 -> F32 -> F64
            continue;
        }
        break;
    }
    const int nchunks = (int)chunks_of(n);
    HIPCHK(ws.partial.ensure((size_t)nchunks * m * m * 8), "alloc partials");
    HIPCHK(launch_charge_partials(X, npad, dcond, n, m, ws.partial.as<double>(), nchunks, st), "charges");
    HIPCHK(launch_charge_finish(ws.partial.as<double>(), nchunks, m, eps_r * kEps0 * lu, dC, st), "charges");
    HIPCHK(end_segment(), "graph");
    HIPCHK(hipEventRecord(ws.ev[3], st), "hipEventRecord");
    HIPCHK(hipMemcpyAsync(&rbk->serr, ws.sync.err, 4, hipMemcpyDeviceToHost, st), "D2H solve flag");
    if (hC) HIPCHK(hipMemcpyAsync(rbk->C, dC, sizeof(double) * m * m, hipMemcpyDeviceToHost, st), "D2H C");
    HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (rbk->perr) {
        set_error("Cholesky: a panel wait exceeded its poll limit");
        return GBEM_EDEVICE;
    }
    if (dtype == GBEM_F64 && rbk->info != 0) {
        set_error("Cholesky: non-positive pivot at row " + std::to_string(rbk->info - 1));
        return GBEM_ENOTPD;
    }
    if (rbk->serr) {
        set_error("triangular solve: a block wait exceeded its poll limit");
        return GBEM_EDEVICE;
    }
    if (hC) memcpy(hC, rbk->C, sizeof(double) * m * m);
    if (rep) {
        float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
        (void)hipEventElapsedTime(&t01, ws.ev[0], ws.ev[1]);
        (void)hipEventElapsedTime(&t12, ws.ev[1], ws.ev[2]);
        (void)hipEventElapsedTime(&t23, ws.ev[2], ws.ev[3]);
        (void)hipEventElapsedTime(&t03, ws.ev[0], ws.ev[3]);
        rep->t_assemble_ms = t01;
        rep->t_factor_ms = t12;
        rep->t_solve_ms = t23;
        rep->t_total_ms = t03;
        rep->residual = resid;
        rep->refine_iters = iters;
        rep->factor_used = dtype;
        const CholShape sh = chol_shape(dtype, npad);
        rep->outer_width = sh.outer_width;
        rep->super_panels = sh.super_panels;
        rep->graph_used = graph_used;
        rep->graph_instantiated = graph_inst;
        pf.collect(rep);
    }
    return GBEM_OK;
}

static double asym_of(const double *C, int m)
{
    double mx = 0.0, d = 0.0;
    for (int i = 0; i < m * m; ++i) mx = std::max(mx, fabs(C[i]));
    for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) d = std::max(d, fabs(C[k * m + l] - C[l * m + k]));
    return mx > 0 ? d / mx : 0.0;
}

// ------------------------------------------------------------------------
// Scratch of the no-allocation entry point (gbem_extract_device_noalloc).
// One static device array per GPU: the loader gives every device that loads
// the library its own copy, held until the process ends.  In host code the
// name `scratch` is only a host-side stand-in; its device address on a GPU
// comes from hipGetSymbolAddress with that GPU current, taken once per device
// when the first context on it is created (noalloc_setup), and only that
// address is ever handed to kernels or copies.
// ------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// largest padded order whose FP64 matrix alone fits the scratch
constexpr int64_t kNoAllocMaxPad = 5632;
static_assert((size_t)kNoAllocMaxPad * kNoAllocMaxPad * 8 <= kNoAllocBytes &&
                  (size_t)(kNoAllocMaxPad + kPad) * (kNoAllocMaxPad + kPad) * 8 > kNoAllocBytes,
              "kNoAllocMaxPad must be the largest padded order with an FP64 matrix inside the scratch");

struct NoAllocDev {
    std::mutex mu;          // calls on this device take turns: they share the array
    void *ptr = nullptr;    // device address of `scratch` on this device
    Arena arena;
    Workspace ws;           // every buffer borrowed from the arena; events, pinned readback and
                            // the factor's event pool created at set-up; no stream of its own
                            // (the look-ahead runs on the caller's stream: a stream more per
                            // process would share the GPU's few hardware queues with the
                            // serving workers' streams)
};
static std::mutex g_noalloc_mu;
static std::vector<NoAllocDev *> g_noalloc;   // by device; entries live until the process ends

// Called by gbem_create with `device` current.
static hipError_t noalloc_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if ((int)g_noalloc.size() <= device) g_noalloc.resize(device + 1, nullptr);
    if (g_noalloc[device]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    NoAllocDev *d = new NoAllocDev();
    d->ptr = ptr;
    d->arena.base = static_cast<unsigned char *>(ptr);
    d->arena.size = kNoAllocBytes;
    d->ws.each([&](DevBuf &b) { b.arena = &d->arena; });
    if ((e = d->ws.init_events()) != hipSuccess) {
        delete d;
        return e;
    }
    d->ws.lookahead_on_main = true;
    // the factorisation's event pool: two events per outer panel of the
    // largest order that fits, with room to spare
    for (int64_t k = 0; k < 4 * (kNoAllocMaxPad / kNB) + 8; ++k) {
        hipEvent_t x;
        if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming | hipEventDisableSystemFence)) != hipSuccess) {
            delete d;
            return e;
        }
        d->ws.fev.push_back(x);
    }
    g_noalloc[device] = d;
    return hipSuccess;
}

}  // namespace gbem

using namespace gbem;

// ------------------------------------------------------------------------
// serving loop
// ------------------------------------------------------------------------
struct gbem_job {
    gbem_ctx *ctx = nullptr;
    std::vector<double> lo, hi, C;
    std::vector<int32_t> cond;
    int n = 0, m = 0;
    double eps_r = 1, lu = 1;
    gbem_opts opts{};
    size_t need = 0;                                  // footprint in an empty workspace
    std::array<size_t, Workspace::kBuffers> needs{};   // per workspace buffer
    int state = 0;   // 0 queued, 1 running, 2 done
    gbem_status status = GBEM_OK;
    gbem_report rep{};
    std::string err;
    std::mutex mu;
    std::condition_variable cv;
};

struct Worker {
    std::thread th;
    hipStream_t stream = nullptr;
    Workspace ws;
    gbem_job *job = nullptr;
    bool busy = false;
    size_t held = 0;    // device bytes this worker may hold while busy (set at dispatch)
    size_t bytes = 0;   // device bytes its workspace holds (updated at each job's end and release)
};

struct gbem_ctx {
    int device = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    Workspace ws;
    std::mutex call_mu;   // serialises the synchronous entry points

    // serving state
    std::mutex mu;
    std::condition_variable cv_sched, cv_work;
    std::deque<gbem_job *> queue;
    std::vector<Worker *> workers;
    std::thread sched;
    bool started = false, stopping = false;
    size_t reserved = 0, peak = 0;
    size_t peak_held = 0;   // largest sum of the workspaces' real sizes seen at a job's end
    int64_t done = 0;

    // lanes of gbem_extract_dielectric_partitioned: a workspace and a stream
    // each, created on first use (under call_mu)
    std::vector<std::unique_ptr<Workspace>> lane_ws;
    std::vector<hipStream_t> lane_st;
};

static constexpr int kWorkers = 4;

static void worker_main(gbem_ctx *ctx, Worker *w)
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        gbem_job *j;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            ctx->cv_work.wait(lk, [&] { return ctx->stopping || w->job != nullptr; });
            if (!w->job && ctx->stopping) return;
            j = w->job;
            // a job that starts beside others (or with more queued) overlaps
            // with their kernels; one that starts alone overlaps its own
            // factorisation's panel chain with the trailing updates on a
            // second stream.  Both orders give the same result.  (Measured on
            // the 256-job stream: one look-ahead stream per busy worker,
            // 9 streams on the device's 4 hardware queues, lowered saturation
            // from 376 to 332 jobs/s.)
            bool company = !ctx->queue.empty();
            for (Worker *c : ctx->workers) company = company || (c != w && c->busy);
            w->ws.lookahead_on_main = company;
        }
        gbem_status st = GBEM_OK;
        gbem_report rep{};
        std::vector<double> C(j->m * j->m);
        {
            double *dC = nullptr;
            hipError_t e = hipSuccess;
            e = w->ws.lo.ensure(sizeof(double) * 3 * j->n);
            if (e == hipSuccess) e = w->ws.hi.ensure(sizeof(double) * 3 * j->n);
            if (e == hipSuccess) e = w->ws.cond.ensure(sizeof(int32_t) * j->n);
            if (e == hipSuccess) e = w->ws.C.ensure(sizeof(double) * j->m * j->m);
            if (e == hipSuccess)
                e = hipMemcpyAsync(w->ws.lo.p, j->lo.data(), sizeof(double) * 3 * j->n, hipMemcpyHostToDevice, w->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(w->ws.hi.p, j->hi.data(), sizeof(double) * 3 * j->n, hipMemcpyHostToDevice, w->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(w->ws.cond.p, j->cond.data(), sizeof(int32_t) * j->n, hipMemcpyHostToDevice,
                                   w->stream);
            if (e != hipSuccess) {
                st = dev_fail(e, "serving: upload");
            } else {
                dC = w->ws.C.as<double>();
                st = run_pipeline(w->ws, w->stream, j->n, j->m, w->ws.lo.as<double>(), w->ws.hi.as<double>(),
                                  w->ws.cond.as<int32_t>(), j->eps_r, j->lu, j->opts, dC, &rep, Stop::kFull,
                                  C.data());
            }
        }
        if (st == GBEM_OK) rep.asym = asym_of(C.data(), j->m);
        const size_t held_now = w->ws.bytes();   // only this thread touches a busy workspace
        const size_t need = j->need;
        std::string err = st != GBEM_OK ? std::string(gbem_last_error()) : std::string();
        // the context's statistics first, then the job's completion: a caller
        // woken by gbem_wait already sees this job counted
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            w->job = nullptr;
            w->busy = false;
            w->bytes = held_now;
            size_t t = 0;
            for (Worker *c : ctx->workers) t += c->bytes;
            ctx->peak_held = std::max(ctx->peak_held, t);
            ctx->reserved -= need;
            ctx->done += 1;
        }
        ctx->cv_sched.notify_all();
        {
            std::lock_guard<std::mutex> lk(j->mu);
            j->status = st;
            j->rep = rep;
            j->C.swap(C);
            if (st != GBEM_OK) j->err = err;
            j->state = 2;
            // notified under the job's lock: its owner cannot free it before
            // this thread lets go of the lock, and nothing of j is touched after
            j->cv.notify_all();
        }
    }
}

// Admission (admission.h): the device memory held by all worker workspaces
// never exceeds the budget (the near list aside, which is estimated before
// its size is known).  This adapter gives the policy the live queue and
// workers; it runs with ctx->mu held, which release_idle gives up while it
// frees memory (hipFree may wait for the device, and workers finishing a job
// need the lock); only this thread dispatches, so an idle worker stays idle
// meanwhile.
struct LivePool {
    gbem_ctx *ctx;
    std::unique_lock<std::mutex> &lk;
    size_t queue_size() const { return ctx->queue.size(); }
    int first_idle() const
    {
        for (size_t i = 0; i < ctx->workers.size(); ++i)
            if (!ctx->workers[i]->busy) return (int)i;
        return -1;
    }
    // idle workspaces are only touched by this thread; busy ones are bounded
    // by what was recorded when they were dispatched
    size_t others(int w) const
    {
        size_t t = 0;
        for (size_t i = 0; i < ctx->workers.size(); ++i) {
            const Worker *c = ctx->workers[i];
            if ((int)i != w) t += c->busy ? std::max(c->held, c->bytes) : c->bytes;
        }
        return t;
    }
    // each buffer grows to the job's need or keeps its larger capacity
    size_t grown(int w, size_t qi) const { return grown_bytes(ctx->workers[w]->ws, ctx->queue[qi]->needs); }
    bool release_idle(size_t qi)
    {
        gbem_job *j = ctx->queue[qi];
        std::vector<Worker *> idle;
        for (Worker *c : ctx->workers)
            if (!c->busy && c->bytes > 0) idle.push_back(c);
        lk.unlock();
        for (Worker *c : idle) c->ws.release_all();
        lk.lock();
        for (Worker *c : idle) c->bytes = 0;
        // a worker that finished meanwhile is idle now and holds its last
        // job's workspace: others() counts it on the next call
        return ctx->queue.size() > qi && ctx->queue[qi] == j;
    }
    void dispatch(size_t qi, int wi, size_t mine, size_t total)
    {
        gbem_job *j = ctx->queue[qi];
        Worker *w = ctx->workers[wi];
        ctx->queue.erase(ctx->queue.begin() + qi);
        {
            std::lock_guard<std::mutex> jl(j->mu);
            j->state = 1;
        }
        w->busy = true;
        w->job = j;
        w->held = mine;
        ctx->reserved += j->need;
        ctx->peak = std::max(ctx->peak, total);
    }
};

// A job at the head of the queue that does not fit may be passed by jobs
// that do for up to one second.
static void sched_main(gbem_ctx *ctx)
{
    (void)hipSetDevice(ctx->device);
    auto head_since = std::chrono::steady_clock::now();
    gbem_job *head_seen = nullptr;
    std::unique_lock<std::mutex> lk(ctx->mu);
    LivePool pool{ctx, lk};
    for (;;) {
        if (ctx->stopping && ctx->queue.empty()) break;
        bool dispatched = false;
        if (!ctx->queue.empty()) {
            if (ctx->queue.front() != head_seen) {
                head_seen = ctx->queue.front();
                head_since = std::chrono::steady_clock::now();
            }
            const bool head_starving = std::chrono::steady_clock::now() - head_since > std::chrono::seconds(1);
            dispatched = admit_one(pool, ctx->budget, head_starving);
        }
        if (dispatched) {
            ctx->cv_work.notify_all();
            continue;
        }
        ctx->cv_sched.wait_for(lk, std::chrono::milliseconds(50));
    }
}

static void start_server(gbem_ctx *ctx)
{
    if (ctx->started) return;
    for (int i = 0; i < kWorkers; ++i) {
        Worker *w = new Worker();
        (void)hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
        ctx->workers.push_back(w);
    }
    for (Worker *w : ctx->workers) w->th = std::thread(worker_main, ctx, w);
    ctx->sched = std::thread(sched_main, ctx);
    ctx->started = true;
}

// ------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------
extern "C" const char *gbem_version(void) { return "gbem-mi355x 0.1 (gfx950)"; }

extern "C" const char *gbem_status_str(gbem_status s)
{
    switch (s) {
    case GBEM_OK: return "ok";
    case GBEM_EINVAL: return "invalid argument";
    case GBEM_ENOMEM: return "out of device memory or HBM budget";
    case GBEM_EDEVICE: return "HIP device error";
    case GBEM_ENOTPD: return "matrix not positive definite";
    case GBEM_ENOCONV: return "iterative refinement did not converge";
    case GBEM_EBUSY: return "busy";
    case GBEM_ETIMEOUT: return "timed out";
    }
    return "unknown status";
}

extern "C" const char *gbem_last_error(void) { return t_err.c_str(); }

extern "C" void gbem_default_opts(gbem_opts *o)
{
    if (!o) return;
    o->far_order = 3;
    o->near_eta = 2.0;
    o->far_dtype = GBEM_F64;
    o->factor_dtype = GBEM_F64;
    o->refine_tol = 1e-6;
    o->max_refine = 30;
    o->profile = 0;
    o->graph = 0;
}

extern "C" gbem_status gbem_create(int device, size_t budget, gbem_ctx **out)
{
    if (!out) {
        set_error("gbem_create: out is NULL");
        return GBEM_EINVAL;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device < 0 || device >= count) {
        set_error("gbem_create: no such HIP device");
        return GBEM_EDEVICE;
    }
    HIPCHK(hipSetDevice(device), "hipSetDevice");
    tuning_autoload();
    gbem_ctx *c = new gbem_ctx();
    c->device = device;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        budget = (size_t)(0.9 * (double)fr);
    }
    c->budget = budget;
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return dev_fail(e, "hipStreamCreate");
    }
    if ((e = noalloc_setup(device)) != hipSuccess) {
        (void)hipStreamDestroy(c->stream);
        delete c;
        return dev_fail(e, "scratch of the no-allocation entry point (hipGetSymbolAddress)");
    }
    *out = c;
    return GBEM_OK;
}

extern "C" gbem_status gbem_destroy(gbem_ctx *ctx)
{
    if (!ctx) return GBEM_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->started) {
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->stopping = true;
        }
        ctx->cv_sched.notify_all();
        ctx->sched.join();
        ctx->cv_work.notify_all();
        for (Worker *w : ctx->workers) {
            w->th.join();
            (void)hipStreamDestroy(w->stream);
            delete w;
        }
    }
    for (hipStream_t st : ctx->lane_st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    ctx->lane_ws.clear();
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GBEM_OK;
}

static gbem_status upload_mesh(gbem_ctx *ctx, const gbem_mesh *mesh)
{
    Workspace &ws = ctx->ws;
    const int n = mesh->n_panels;
    HIPCHK(ws.lo.ensure(sizeof(double) * 3 * n), "alloc mesh");
    HIPCHK(ws.hi.ensure(sizeof(double) * 3 * n), "alloc mesh");
    HIPCHK(ws.cond.ensure(sizeof(int32_t) * n), "alloc mesh");
    HIPCHK(hipMemcpyAsync(ws.lo.p, mesh->lo, sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream), "H2D");
    HIPCHK(hipMemcpyAsync(ws.hi.p, mesh->hi, sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream), "H2D");
    HIPCHK(hipMemcpyAsync(ws.cond.p, mesh->conductor, sizeof(int32_t) * n, hipMemcpyHostToDevice, ctx->stream),
           "H2D");
    return GBEM_OK;
}

// Mesh header and options are checked before the context, so argument
// errors are reported the same way with or without a device.
static gbem_status check_args(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, gbem_opts &o)
{
    std::string why;
    if (!mesh_header_ok(mesh, why)) {
        set_error(why);
        return GBEM_EINVAL;
    }
    if (opts) o = *opts; else gbem_default_opts(&o);
    if (!opts_ok(o, why)) {
        set_error(why);
        return GBEM_EINVAL;
    }
    if (!ctx) {
        set_error("context is NULL");
        return GBEM_EINVAL;
    }
    return GBEM_OK;
}

extern "C" gbem_status gbem_extract(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                    double *C_out, gbem_report *rep)
{
    gbem_opts o;
    gbem_status s = check_args(ctx, mesh, opts, o);
    if (s != GBEM_OK) return s;
    if (!C_out) {
        set_error("C_out is NULL");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    if ((s = upload_mesh(ctx, mesh)) != GBEM_OK) return s;
    const int m = mesh->n_conductors;
    HIPCHK(ctx->ws.C.ensure(sizeof(double) * m * m), "alloc C");
    gbem_report r{};
    std::vector<double> C(m * m);
    s = run_pipeline(ctx->ws, ctx->stream, mesh->n_panels, m, ctx->ws.lo.as<double>(), ctx->ws.hi.as<double>(),
                     ctx->ws.cond.as<int32_t>(), mesh->eps_r, mesh->length_unit_m, o, ctx->ws.C.as<double>(),
                     &r, Stop::kFull, C.data());
    if (s != GBEM_OK) {
        if (rep) *rep = r;
        return s;
    }
    memcpy(C_out, C.data(), sizeof(double) * m * m);
    r.asym = asym_of(C.data(), m);
    if (rep) *rep = r;
    return GBEM_OK;
}

extern "C" gbem_status gbem_extract_device(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                           double *C_out_device, void *stream, gbem_report *rep)
{
    gbem_opts o;
    gbem_status s = check_args(ctx, mesh, opts, o);
    if (s != GBEM_OK) return s;
    if (!C_out_device) {
        set_error("C_out_device is NULL");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    gbem_report r{};
    const int m = mesh->n_conductors;
    std::vector<double> C(rep ? m * m : 0);   // host copy only for the report's asymmetry
    s = run_pipeline(ctx->ws, st, mesh->n_panels, m, mesh->lo, mesh->hi, mesh->conductor, mesh->eps_r,
                     mesh->length_unit_m, o, C_out_device, &r, Stop::kFull, rep ? C.data() : nullptr);
    if (s == GBEM_OK && rep) r.asym = asym_of(C.data(), m);
    if (rep) *rep = r;
    return s;
}

extern "C" gbem_status gbem_extract_device_noalloc(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                                   double *C_out_device, void *stream, gbem_report *rep)
{
    gbem_opts o;
    gbem_status s = check_args(ctx, mesh, opts, o);
    if (s != GBEM_OK) return s;
    if (!C_out_device) {
        set_error("C_out_device is NULL");
        return GBEM_EINVAL;
    }
    if (o.profile != 0) {
        set_error("gbem_extract_device_noalloc: opts->profile must be 0 (the timing events would be created "
                  "during the call)");
        return GBEM_EINVAL;
    }
    if (o.graph != 0) {
        set_error("gbem_extract_device_noalloc: opts->graph must be 0 (instantiating a graph allocates)");
        return GBEM_EINVAL;
    }
    const int n = mesh->n_panels, m = mesh->n_conductors;
    const int64_t npad = round_up(n, kPad);
    // the buffers whose size the mesh fixes, for the requested factor and
    // every fallback level (the near list is checked once its size is known)
    size_t fixed = 0;
    for (size_t b : buffer_needs(n, m, o.factor_dtype, false, false)) fixed += b;
    if (npad > kNoAllocMaxPad || fixed > kNoAllocBytes) {
        set_error("gbem_extract_device_noalloc: a mesh of " + std::to_string(n) + " panels needs about " +
                  std::to_string(fixed >> 20) + " MiB of scratch; the no-allocation entry point has " +
                  std::to_string(kNoAllocBytes >> 20) + " MiB per GPU (use gbem_extract_device)");
        return GBEM_ENOMEM;
    }
    NoAllocDev *d = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (ctx->device < (int)g_noalloc.size()) d = g_noalloc[ctx->device];
    }
    if (!d) {
        set_error("gbem_extract_device_noalloc: the context's device has no scratch set up");
        return GBEM_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(d->mu);
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    // hand the whole array back to the arena: every buffer is carved again,
    // and the triangular solves' flags are zeroed again when carved
    d->ws.release_all();
    d->arena.reset();
    d->ws.sync_npad = -1;
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    gbem_report r{};
    double hC[kMaxRhs * kMaxRhs];
    s = run_pipeline(d->ws, st, n, m, mesh->lo, mesh->hi, mesh->conductor, mesh->eps_r, mesh->length_unit_m, o,
                     C_out_device, &r, Stop::kFull, hC);
    if (s == GBEM_ENOMEM && d->arena.exhausted)
        set_error("gbem_extract_device_noalloc: the " + std::to_string(kNoAllocBytes >> 20) +
                  " MiB scratch cannot hold this job (" + gbem_last_error() +
                  "); use gbem_extract_device");
    if (s == GBEM_OK) r.asym = asym_of(hC, m);
    if (rep) *rep = r;
    return s;
}

extern "C" gbem_status gbem_submit(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, gbem_job **out)
{
    gbem_opts o;
    gbem_status s = check_args(ctx, mesh, opts, o);
    if (s != GBEM_OK) return s;
    if (!out) {
        set_error("out is NULL");
        return GBEM_EINVAL;
    }
    gbem_job *j = new gbem_job();
    j->ctx = ctx;
    j->n = mesh->n_panels;
    j->m = mesh->n_conductors;
    j->lo.assign(mesh->lo, mesh->lo + 3 * (size_t)j->n);
    j->hi.assign(mesh->hi, mesh->hi + 3 * (size_t)j->n);
    j->cond.assign(mesh->conductor, mesh->conductor + j->n);
    j->eps_r = mesh->eps_r;
    j->lu = mesh->length_unit_m;
    j->opts = o;
    j->needs = buffer_needs(j->n, j->m, o.factor_dtype, true, true);
    j->need = footprint(j->n, j->m, o.factor_dtype);
    if (j->need > ctx->budget) {
        delete j;
        set_error("job footprint exceeds the HBM budget of the context");
        return GBEM_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        start_server(ctx);
        ctx->queue.push_back(j);
    }
    ctx->cv_sched.notify_all();
    *out = j;
    return GBEM_OK;
}

extern "C" gbem_status gbem_poll(gbem_job *j)
{
    if (!j) return GBEM_EINVAL;
    std::lock_guard<std::mutex> lk(j->mu);
    if (j->state != 2) return GBEM_EBUSY;
    return j->status;
}

extern "C" gbem_status gbem_wait(gbem_job *j, double timeout_s, double *C_out, gbem_report *rep)
{
    if (!j) return GBEM_EINVAL;
    std::unique_lock<std::mutex> lk(j->mu);
    if (timeout_s < 0) {
        j->cv.wait(lk, [&] { return j->state == 2; });
    } else if (!j->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return j->state == 2; })) {
        set_error("gbem_wait: timed out");
        return GBEM_ETIMEOUT;
    }
    if (j->status != GBEM_OK) {
        set_error(j->err);
        if (rep) *rep = j->rep;
        return j->status;
    }
    if (C_out) memcpy(C_out, j->C.data(), sizeof(double) * j->m * j->m);
    if (rep) *rep = j->rep;
    return GBEM_OK;
}

extern "C" void gbem_job_free(gbem_job *j)
{
    if (!j) return;
    {
        std::unique_lock<std::mutex> lk(j->mu);
        j->cv.wait(lk, [&] { return j->state == 2; });
    }
    delete j;
}

extern "C" gbem_status gbem_server_stats(gbem_ctx *ctx, int64_t *jobs_done, size_t *peak_reserved_bytes,
                                         size_t *peak_held_bytes)
{
    if (!ctx) return GBEM_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (jobs_done) *jobs_done = ctx->done;
    if (peak_reserved_bytes) *peak_reserved_bytes = ctx->peak;
    if (peak_held_bytes) *peak_held_bytes = ctx->peak_held;
    return GBEM_OK;
}

// ---- stage entry points ----------------------------------------------------
extern "C" gbem_status gbem_near_list(gbem_ctx *ctx, const gbem_mesh *mesh, double near_eta, int64_t *row_ptr,
                                      int32_t *col, int64_t col_capacity, int64_t *nnz)
{
    gbem_opts o;
    gbem_default_opts(&o);
    o.near_eta = near_eta;
    gbem_status s = check_args(ctx, mesh, &o, o);
    if (s != GBEM_OK) return s;
    if (!row_ptr || !nnz) {
        set_error("row_ptr and nnz are required");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    if ((s = upload_mesh(ctx, mesh)) != GBEM_OK) return s;
    Workspace &ws = ctx->ws;
    const int n = mesh->n_panels;
    HIPCHK(ws.cnt.ensure(sizeof(int64_t) * n), "alloc");
    HIPCHK(ws.rowptr.ensure(sizeof(int64_t) * (n + 1)), "alloc");
    HIPCHK(ws.nmask.ensure(sizeof(uint64_t) * (size_t)n * near_mask_words(n)), "alloc");
    const double eta2 = near_eta * near_eta;
    HIPCHK(launch_near_count(ws.lo.as<double>(), ws.hi.as<double>(), n, eta2, ws.cnt.as<int64_t>(),
                             ws.nmask.as<uint64_t>(), ctx->stream), "near_count");
    HIPCHK(launch_exclusive_scan(ws.cnt.as<int64_t>(), n, ws.rowptr.as<int64_t>(), ctx->stream), "scan");
    HIPCHK(hipMemcpyAsync(row_ptr, ws.rowptr.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, ctx->stream), "D2H");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    *nnz = row_ptr[n];
    if (!col) return GBEM_OK;
    if (col_capacity < *nnz) {
        set_error("col_capacity is smaller than the number of near pairs");
        return GBEM_EINVAL;
    }
    HIPCHK(ws.nrow.ensure(sizeof(int32_t) * std::max<int64_t>(*nnz, 1)), "alloc");
    HIPCHK(ws.ncol.ensure(sizeof(int32_t) * std::max<int64_t>(*nnz, 1)), "alloc");
    HIPCHK(launch_near_fill(ws.nmask.as<uint64_t>(), n, ws.rowptr.as<int64_t>(), ws.nrow.as<int32_t>(),
                            ws.ncol.as<int32_t>(), ctx->stream), "near_fill");
    HIPCHK(hipMemcpyAsync(col, ws.ncol.p, sizeof(int32_t) * *nnz, hipMemcpyDeviceToHost, ctx->stream), "D2H");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    return GBEM_OK;
}

static gbem_status assemble_common(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, gbem_report *r,
                                   Stop stop = Stop::kAssembled)
{
    gbem_opts o;
    gbem_status s = check_args(ctx, mesh, opts, o);
    if (s != GBEM_OK) return s;
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    if ((s = upload_mesh(ctx, mesh)) != GBEM_OK) return s;
    return run_pipeline(ctx->ws, ctx->stream, mesh->n_panels, mesh->n_conductors, ctx->ws.lo.as<double>(),
                        ctx->ws.hi.as<double>(), ctx->ws.cond.as<int32_t>(), mesh->eps_r, mesh->length_unit_m, o,
                        nullptr, r, stop);
}

extern "C" gbem_status gbem_assemble(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, double *A_out)
{
    if (!A_out) {
        set_error("A_out is NULL");
        return GBEM_EINVAL;
    }
    if (!ctx) return GBEM_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    gbem_report r{};
    gbem_status s = assemble_common(ctx, mesh, opts, &r);
    if (s != GBEM_OK) return s;
    const int n = mesh->n_panels;
    const int64_t npad = round_up(n, kPad);
    // A is symmetric: its column-major n x n block read row by row is the row-major matrix
    HIPCHK(hipMemcpy2DAsync(A_out, sizeof(double) * n, ctx->ws.A.p, sizeof(double) * npad, sizeof(double) * n, n,
                            hipMemcpyDeviceToHost, ctx->stream), "D2H A");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    return GBEM_OK;
}

extern "C" gbem_status gbem_assemble_sample(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, int64_t m,
                                            const int32_t *ii, const int32_t *jj, double *out)
{
    if (!ctx || m < 0 || (m > 0 && (!ii || !jj || !out))) {
        set_error("gbem_assemble_sample: bad arguments");
        return GBEM_EINVAL;
    }
    const int n = mesh ? mesh->n_panels : 0;
    for (int64_t k = 0; k < m; ++k)
        if (ii[k] < 0 || ii[k] >= n || jj[k] < 0 || jj[k] >= n) {
            set_error("gbem_assemble_sample: index out of range");
            return GBEM_EINVAL;
        }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    gbem_report r{};
    gbem_status s = assemble_common(ctx, mesh, opts, &r);
    if (s != GBEM_OK || m == 0) return s;
    Workspace &ws = ctx->ws;
    DevBuf di, dj, dout;
    HIPCHK(di.ensure(sizeof(int32_t) * m), "alloc");
    HIPCHK(dj.ensure(sizeof(int32_t) * m), "alloc");
    HIPCHK(dout.ensure(sizeof(double) * m), "alloc");
    HIPCHK(hipMemcpyAsync(di.p, ii, sizeof(int32_t) * m, hipMemcpyHostToDevice, ctx->stream), "H2D");
    HIPCHK(hipMemcpyAsync(dj.p, jj, sizeof(int32_t) * m, hipMemcpyHostToDevice, ctx->stream), "H2D");
    HIPCHK(launch_gather(ws.A.as<double>(), round_up(n, kPad), di.as<int32_t>(), dj.as<int32_t>(), m,
                         dout.as<double>(), ctx->stream), "gather");
    HIPCHK(hipMemcpyAsync(out, dout.p, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->stream), "D2H");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    di.release();
    dj.release();
    dout.release();
    return GBEM_OK;
}

// m sampled entries of the FP32 factor input F = S A S written by the
// assembly passes (lower triangle: ii[k] >= jj[k])
extern "C" gbem_status gbem_assemble_scaled_sample(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                                   int64_t m, const int32_t *ii, const int32_t *jj, float *out)
{
    if (!ctx || !opts || m < 0 || (m > 0 && (!ii || !jj || !out))) {
        set_error("gbem_assemble_scaled_sample: bad arguments");
        return GBEM_EINVAL;
    }
    if (opts->factor_dtype == GBEM_F64) {
        set_error("gbem_assemble_scaled_sample: an FP64 factor has no scaled FP32 copy");
        return GBEM_EINVAL;
    }
    const int n = mesh ? mesh->n_panels : 0;
    for (int64_t k = 0; k < m; ++k)
        if (jj[k] < 0 || ii[k] < jj[k] || ii[k] >= n) {
            set_error("gbem_assemble_scaled_sample: index out of range or above the diagonal");
            return GBEM_EINVAL;
        }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    gbem_report r{};
    gbem_status s = assemble_common(ctx, mesh, opts, &r, Stop::kScaled);
    if (s != GBEM_OK || m == 0) return s;
    Workspace &ws = ctx->ws;
    DevBuf di, dj, dout;
    HIPCHK(di.ensure(sizeof(int32_t) * m), "alloc");
    HIPCHK(dj.ensure(sizeof(int32_t) * m), "alloc");
    HIPCHK(dout.ensure(sizeof(float) * m), "alloc");
    HIPCHK(hipMemcpyAsync(di.p, ii, sizeof(int32_t) * m, hipMemcpyHostToDevice, ctx->stream), "H2D");
    HIPCHK(hipMemcpyAsync(dj.p, jj, sizeof(int32_t) * m, hipMemcpyHostToDevice, ctx->stream), "H2D");
    HIPCHK(launch_gather(ws.F.as<float>(), round_up(n, kPad), di.as<int32_t>(), dj.as<int32_t>(), m,
                         dout.as<float>(), ctx->stream), "gather");
    HIPCHK(hipMemcpyAsync(out, dout.p, sizeof(float) * m, hipMemcpyDeviceToHost, ctx->stream), "D2H");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    di.release();
    dj.release();
    dout.release();
    return GBEM_OK;
}

static gbem_status chol_common(gbem_ctx *ctx, int32_t n, int32_t dtype, void *A, int64_t lda, int32_t *info,
                               void *stream, int32_t nrhs, void *Bm, int64_t ldb, bool solve)
{
    if (!ctx || n <= 0 || !A || lda < n || dtype < GBEM_F64 || dtype > GBEM_BF16 ||
        (solve && (!Bm || nrhs <= 0 || nrhs > kMaxRhs || ldb < n))) {
        set_error("cholesky: bad arguments");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
    Workspace &ws = ctx->ws;
    const int64_t npad = round_up(n, kPad);
    const size_t es = dtype == GBEM_F64 ? 8 : 4;
    DevBuf &Ap = dtype == GBEM_F64 ? ws.A : ws.F;
    HIPCHK(Ap.ensure((size_t)npad * npad * es), "alloc");
    HIPCHK(ws.Winv.ensure(chol_winv_bytes(dtype, npad)), "alloc");
    HIPCHK(ws.Pw.ensure(chol_panel_bytes(dtype, npad)), "alloc");
    HIPCHK(ws.P16.ensure(std::max<size_t>(chol_panel16_bytes(dtype, npad), 64)), "alloc");
    HIPCHK(ws.flags.ensure(64), "alloc");
    HIPCHK(hipMemcpy2DAsync(Ap.p, es * npad, A, es * lda, es * n, n, hipMemcpyDeviceToDevice, st), "copy in");
    HIPCHK(launch_identity_pad(Ap.p, npad, n, (int)npad, dtype == GBEM_F64, st), "pad");
    if (!solve) {
        HIPCHK(hipMemsetAsync(ws.flags.p, 0, 64, st), "memset");
        HIPCHK(ws.ensure_side(), "side stream");
        HIPCHK(chol_factor(dtype, npad, Ap.p, npad, ws.Winv.p, ws.Pw.p, ws.P16.p, ws.flags.as<int32_t>() + 1, st,
                           ws.side, ws.fev),
               "cholesky");
        int32_t ie[2] = {0, 0};   // pivot status, panel wait error
        HIPCHK(hipMemcpyAsync(ie, ws.flags.as<int32_t>() + 1, 8, hipMemcpyDeviceToHost, st), "D2H");
        HIPCHK(hipStreamSynchronize(st), "sync");
        if (ie[1]) {
            set_error("Cholesky: a panel wait exceeded its poll limit");
            return GBEM_EDEVICE;
        }
        int32_t inf = ie[0];
        if (info) *info = inf;
        if (inf > n) inf = 0;   // a pivot in the identity padding cannot fail
        if (inf != 0) {
            set_error("Cholesky: non-positive pivot at row " + std::to_string(inf - 1));
            return GBEM_ENOTPD;
        }
        HIPCHK(hipMemcpy2DAsync(A, es * lda, Ap.p, es * npad, es * n, n, hipMemcpyDeviceToDevice, st), "copy out");
        HIPCHK(hipStreamSynchronize(st), "sync");
        return GBEM_OK;
    }
    HIPCHK(chol_diag_inverses(dtype, npad, Ap.p, npad, ws.Winv.p, st), "diag inverses");
    HIPCHK(ws.ensure_sync(npad, st), "alloc solve flags");
    HIPCHK(chol_solve_prep(dtype, npad, Ap.p, npad, ws.Winv.p, ws.sync, st), "solve prep");
    HIPCHK(ws.X.ensure((size_t)npad * nrhs * 8), "alloc");
    HIPCHK(hipMemsetAsync(ws.X.p, 0, (size_t)npad * nrhs * 8, st), "memset");
    HIPCHK(hipMemcpy2DAsync(ws.X.p, 8 * npad, Bm, 8 * ldb, 8 * n, nrhs, hipMemcpyDeviceToDevice, st), "copy B");
    HIPCHK(hipMemsetAsync(ws.sync.err, 0, 4, st), "memset");
    HIPCHK(chol_solve(dtype, npad, Ap.p, npad, ws.Winv.p, nrhs, ws.X.as<double>(), npad, ws.sync, st), "solve");
    int32_t serr = 0;
    HIPCHK(hipMemcpyAsync(&serr, ws.sync.err, 4, hipMemcpyDeviceToHost, st), "D2H");
    HIPCHK(hipStreamSynchronize(st), "sync");
    if (serr) {
        set_error("triangular solve: a block wait exceeded its poll limit");
        return GBEM_EDEVICE;
    }
    HIPCHK(hipMemcpy2DAsync(Bm, 8 * ldb, ws.X.p, 8 * npad, 8 * n, nrhs, hipMemcpyDeviceToDevice, st), "copy out");
    HIPCHK(hipStreamSynchronize(st), "sync");
    return GBEM_OK;
}

extern "C" gbem_status gbem_cholesky_device(gbem_ctx *ctx, int32_t n, int32_t dtype, void *A, int64_t lda,
                                            int32_t *info, void *stream)
{
    return chol_common(ctx, n, dtype, A, lda, info, stream, 0, nullptr, 0, false);
}

extern "C" gbem_status gbem_cholesky_solve_device(gbem_ctx *ctx, int32_t n, int32_t dtype, const void *L,
                                                  int64_t lda, int32_t nrhs, void *B, int64_t ldb, void *stream)
{
    return chol_common(ctx, n, dtype, const_cast<void *>(L), lda, nullptr, stream, nrhs, B, ldb, true);
}

extern "C" gbem_status gbem_extract_partitioned(gbem_ctx *ctx, const double *box_lo, const double *box_hi,
                                                const int32_t *box_cond, int32_t n_boxes, int32_t n_conductors,
                                                double eps_r, double length_unit_m, const gbem_partition *rule,
                                                const gbem_opts *opts, double *C_out, int32_t *panels_out,
                                                gbem_report *rep)
{
    if (!ctx || !box_lo || !box_hi || !box_cond || !rule || !C_out || n_boxes <= 0) {
        set_error("gbem_extract_partitioned: null argument or no boxes");
        return GBEM_EINVAL;
    }
    if (n_conductors <= 0 || n_conductors > kMaxRhs) {
        set_error("gbem_extract_partitioned: n_conductors must be 1.." + std::to_string(kMaxRhs));
        return GBEM_EINVAL;
    }
    const int m = n_conductors;
    std::vector<double> C(m * m), Ck(m * m);
    gbem_report tot{};
    // the meshes are independent: they go through the serving loop, which
    // runs up to kWorkers of them at once on streams of their own
    std::vector<gbem_job *> jobs(m, nullptr);
    auto drop = [&](int upto) {
        for (int k = 0; k < upto; ++k)
            if (jobs[k]) gbem_job_free(jobs[k]);
    };
    for (int k = 0; k < m; ++k) {
        gbem_mesh_buf buf{};
        gbem_status s = gbem_mesh_partition(box_lo, box_hi, box_cond, n_boxes, k, rule, &buf);
        if (s != GBEM_OK) {
            drop(k);
            return s;
        }
        const gbem_mesh mesh{buf.n_panels, m, buf.lo, buf.hi, buf.conductor, eps_r, length_unit_m};
        if (panels_out) panels_out[k] = mesh.n_panels;
        s = gbem_submit(ctx, &mesh, opts, &jobs[k]);   // copies the mesh
        gbem_mesh_buf_free(&buf);
        if (s != GBEM_OK) {
            drop(k);
            return s;
        }
    }
    gbem_status first_err = GBEM_OK;
    std::string err_msg;
    for (int k = 0; k < m; ++k) {
        gbem_report r{};
        const gbem_status s = gbem_wait(jobs[k], -1.0, Ck.data(), &r);
        if (s != GBEM_OK) {
            if (first_err == GBEM_OK) {
                first_err = s;
                err_msg = gbem_last_error();
            }
            continue;
        }
        for (int n = 0; n < m; ++n) C[n * m + k] = Ck[n * m + k];   // column k: charges with net k at 1 V
        tot.t_assemble_ms += r.t_assemble_ms;
        tot.t_factor_ms += r.t_factor_ms;
        tot.t_solve_ms += r.t_solve_ms;
        tot.t_total_ms += r.t_total_ms;
        tot.residual = std::max(tot.residual, r.residual);
        tot.refine_iters = std::max(tot.refine_iters, r.refine_iters);
        tot.factor_used = r.factor_used;
        tot.n_near += r.n_near;
        tot.n_panels += r.n_panels;
        for (int c = 0; c < GBEM_K_COUNT; ++c) {
            tot.prof_ms[c] += r.prof_ms[c];
            tot.prof_launches[c] += r.prof_launches[c];
            tot.prof_flops[c] += r.prof_flops[c];
            tot.prof_bytes[c] += r.prof_bytes[c];
        }
    }
    drop(m);
    if (first_err != GBEM_OK) {
        set_error("gbem_extract_partitioned: " + err_msg);
        return first_err;
    }
    memcpy(C_out, C.data(), sizeof(double) * m * m);
    tot.asym = asym_of(C.data(), m);
    if (rep) *rep = tot;
    return GBEM_OK;
}

// ------------------------------------------------------------------------
// Multi-dielectric case (section 4)
// ------------------------------------------------------------------------

// Panel table, near list (near_eta) and the double-layer matrix Q (n x n,
// column-major, ldq = n) of the mesh in ws.lo / ws.hi with conductor ids in
// ws.cond; optionally the single-layer matrix A (FP64 far rule of order p)
// in ws.A (npad x npad).  Returns the near-pair count in *nnz.
// Near/far split of the double-layer integrals inside gbem_extract_dielectric:
// fixed, whatever the single layer's near_eta, since both of its rules were
// verified there (closed form below it; the far rule's error is about 1e-15
// |I_i| at it, while the closed form loses digits with distance).
constexpr double kDlNearEta = 2.0;

// Panel table and the double-layer matrix Q (n x n, column-major, ldq = n) of
// the mesh in ws.lo / ws.hi with conductor ids in ws.cond, near pairs of q_eta
// in closed form; with_A: also the single-layer matrix A (FP64, far rule of
// order p, near pairs of near_eta exact) in ws.A (npad x npad).  *nnz: the
// near pairs of the single layer (with_A) or of Q.
static gbem_status dl_assemble(Workspace &ws, int n, int n_cond, double near_eta, double q_eta, int p, bool with_A,
                               DevBuf &Q, int64_t *nnz, hipStream_t st)
{
    const int64_t npad = round_up(n, kPad);
    HIPCHK(ws.pan.ensure(sizeof(Panel) * n), "alloc panels");
    HIPCHK(ws.flags.ensure(64), "alloc flags");
    HIPCHK(ws.cnt.ensure(sizeof(int64_t) * n), "alloc");
    HIPCHK(ws.rowptr.ensure(sizeof(int64_t) * (n + 1)), "alloc");
    HIPCHK(ws.nmask.ensure(sizeof(uint64_t) * (size_t)n * near_mask_words(n)), "alloc");
    HIPCHK(hipMemsetAsync(ws.flags.p, 0, 64, st), "memset");
    HIPCHK(launch_build_panels(ws.lo.as<double>(), ws.hi.as<double>(), ws.cond.as<int32_t>(), n, n_cond,
                               ws.pan.as<Panel>(), ws.flags.as<int32_t>(), st), "build_panels");
    // the near list of eta into (row, col); the panel check with the first one
    bool checked = false;
    auto near_list = [&](double eta, DevBuf &row, DevBuf &col, int64_t *count) -> gbem_status {
        HIPCHK(launch_near_count(ws.lo.as<double>(), ws.hi.as<double>(), n, eta * eta, ws.cnt.as<int64_t>(),
                                 ws.nmask.as<uint64_t>(), st), "near_count");
        HIPCHK(launch_exclusive_scan(ws.cnt.as<int64_t>(), n, ws.rowptr.as<int64_t>(), st), "scan");
        int64_t cnt = 0;
        int32_t bad = 0;
        HIPCHK(hipMemcpyAsync(&cnt, ws.rowptr.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st), "D2H");
        if (!checked) HIPCHK(hipMemcpyAsync(&bad, ws.flags.p, 4, hipMemcpyDeviceToHost, st), "D2H");
        HIPCHK(hipStreamSynchronize(st), "sync");
        checked = true;
        if (bad) {
            set_error("panel " + std::to_string(bad - 1) +
                      " is not an axis-aligned rectangle with exactly one zero extent");
            return GBEM_EINVAL;
        }
        HIPCHK(row.ensure(sizeof(int32_t) * std::max<int64_t>(cnt, 1)), "alloc");
        HIPCHK(col.ensure(sizeof(int32_t) * std::max<int64_t>(cnt, 1)), "alloc");
        HIPCHK(launch_near_fill(ws.nmask.as<uint64_t>(), n, ws.rowptr.as<int64_t>(), row.as<int32_t>(),
                                col.as<int32_t>(), st), "near_fill");
        *count = cnt;
        return GBEM_OK;
    };
    gbem_status s = GBEM_OK;
    int64_t cnt = 0, qcnt = 0;
    if (with_A) {
        if ((s = near_list(near_eta, ws.nrow, ws.ncol, &cnt)) != GBEM_OK) return s;
        HIPCHK(ws.A.ensure((size_t)npad * npad * 8), "alloc A");
        HIPCHK(ws.semi.ensure(near_semi_bytes(cnt)), "alloc near queue");
        GaussRule rule;
        gauss_legendre_rule(p, &rule);
        HIPCHK(launch_far(ws.pan.as<Panel>(), n, (int)npad, p, rule, GBEM_F64, ws.A.as<double>(), npad, st), "far");
        HIPCHK(launch_near_eval(ws.lo.as<double>(), ws.hi.as<double>(), ws.pan.as<Panel>(), ws.nrow.as<int32_t>(),
                                ws.ncol.as<int32_t>(), cnt, ws.A.as<double>(), npad, ws.semi.as<int32_t>(), st),
               "near_eval");
    }
    const bool same = with_A && q_eta == near_eta;
    if (!same && (s = near_list(q_eta, ws.dl.qrow, ws.dl.qcol, &qcnt)) != GBEM_OK) return s;
    const int32_t *qr = same ? ws.nrow.as<int32_t>() : ws.dl.qrow.as<int32_t>();
    const int32_t *qc = same ? ws.ncol.as<int32_t>() : ws.dl.qcol.as<int32_t>();
    HIPCHK(Q.ensure((size_t)n * n * 8), "alloc Q");
    HIPCHK(launch_double_layer(ws.pan.as<Panel>(), n, qr, qc, same ? cnt : qcnt, Q.as<double>(), n, st),
           "double layer");
    *nnz = with_A ? cnt : qcnt;
    return GBEM_OK;
}

extern "C" gbem_status gbem_assemble_double_layer(gbem_ctx *ctx, int32_t n_panels, const double *lo,
                                                  const double *hi, double near_eta, double *Q_out)
{
    if (!ctx || n_panels <= 0 || !lo || !hi || !Q_out || !(near_eta >= kMinNearEta) || !isfinite(near_eta)) {
        set_error("gbem_assemble_double_layer: null argument, no panels or near_eta < 1e-6");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    Workspace &ws = ctx->ws;
    const int n = n_panels;
    hipStream_t st = ctx->stream;
    HIPCHK(ws.lo.ensure(sizeof(double) * 3 * n), "alloc mesh");
    HIPCHK(ws.hi.ensure(sizeof(double) * 3 * n), "alloc mesh");
    HIPCHK(ws.cond.ensure(sizeof(int32_t) * n), "alloc mesh");
    HIPCHK(hipMemcpyAsync(ws.lo.p, lo, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st), "H2D");
    HIPCHK(hipMemcpyAsync(ws.hi.p, hi, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st), "H2D");
    HIPCHK(hipMemsetAsync(ws.cond.p, 0xff, sizeof(int32_t) * n, st), "memset");   // -1: no conductor
    DevBuf &Q = ws.dl.Q;
    int64_t nnz = 0;
    gbem_status s = dl_assemble(ws, n, 0, near_eta, near_eta, 3, false, Q, &nnz, st);
    if (s != GBEM_OK) return s;
    std::vector<double> tmp((size_t)n * n);
    HIPCHK(hipMemcpyAsync(tmp.data(), Q.p, sizeof(double) * n * n, hipMemcpyDeviceToHost, st), "D2H");
    HIPCHK(hipStreamSynchronize(st), "sync");
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) Q_out[(size_t)i * n + k] = tmp[i + (size_t)k * n];
    return GBEM_OK;
}

// The extraction on the context's workspace and stream (lane == nullptr, the
// synchronous entry: serialised by call_mu) or on a lane's own workspace and
// stream (the caller holds call_mu and has made the device current).
struct Lane {
    Workspace *ws;
    hipStream_t st;
};
static gbem_status dielectric_run(gbem_ctx *ctx, const Lane *lane, const gbem_dmesh *mesh, const gbem_opts *opts,
                                  double *C_out, gbem_report *rep)
{
    const auto t_start = std::chrono::steady_clock::now();
    if (!mesh || !C_out || !mesh->lo || !mesh->hi || !mesh->kind || !mesh->conductor || !mesh->region_plus ||
        !mesh->region_minus || !mesh->eps_r || mesh->n_panels <= 0 || mesh->n_conductors <= 0 ||
        mesh->n_conductors > kMaxRhs || mesh->n_regions <= 0 || !(mesh->length_unit_m > 0.0)) {
        set_error("gbem_extract_dielectric: null argument, no panels, or n_conductors outside 1..64, or no region");
        return GBEM_EINVAL;
    }
    gbem_opts o;
    if (opts) o = *opts; else gbem_default_opts(&o);
    std::string why;
    if (!opts_ok(o, why)) {
        set_error("gbem_extract_dielectric: " + why);
        return GBEM_EINVAL;
    }
    const int n = mesh->n_panels, M = mesh->n_conductors, R = mesh->n_regions;
    for (int a = 0; a < R; ++a)
        if (!(mesh->eps_r[a] > 0.0) || !isfinite(mesh->eps_r[a])) {
            set_error("gbem_extract_dielectric: eps_r of region " + std::to_string(a) + " must be > 0");
            return GBEM_EINVAL;
        }
    // unknown slots and equations (region-major, panels in order), as in the
    // section 4.1 system: q on conductor, Dirichlet and interface panels, u on
    // Neumann and interface panels
    std::vector<int32_t> u_slot(n, -1), q_slot(n, -1), cond(n, -1), eq_reg, eq_pan;
    int nu = 0;
    for (int i = 0; i < n; ++i) {
        const int k = mesh->kind[i], rp = mesh->region_plus[i], rm = mesh->region_minus[i];
        const bool rp_ok = rp >= -1 && rp < R, rm_ok = rm >= -1 && rm < R;
        const int sides = (rp >= 0) + (rm >= 0);
        bool ok = rp_ok && rm_ok && k >= GBEM_PANEL_CONDUCTOR && k <= GBEM_PANEL_INTERFACE;
        if (ok && k == GBEM_PANEL_INTERFACE) ok = sides == 2 && rp != rm;
        else if (ok) ok = sides == 1;
        if (ok && k == GBEM_PANEL_CONDUCTOR) ok = mesh->conductor[i] >= 0 && mesh->conductor[i] < M;
        if (!ok) {
            set_error("gbem_extract_dielectric: panel " + std::to_string(i) +
                      ": kind, regions or conductor id inconsistent (conductor, Dirichlet and Neumann panels bound "
                      "one region, interface panels two different ones)");
            return GBEM_EINVAL;
        }
        if (k == GBEM_PANEL_CONDUCTOR) cond[i] = mesh->conductor[i];
    }
    // unknowns ordered by the pair (lower, upper region) of their panel, so
    // that the unknowns of one region's boundary lie in a narrow slot range
    // (contiguous for layered regions); per panel q first, then u
    auto lower_region = [&](int i) {
        const int a = mesh->region_plus[i], b = mesh->region_minus[i];
        return a < 0 ? b : (b < 0 ? a : std::min(a, b));
    };
    auto upper_region = [&](int i) { return std::max(mesh->region_plus[i], mesh->region_minus[i]); };
    std::vector<int> porder(n);
    for (int i = 0; i < n; ++i) porder[i] = i;
    std::stable_sort(porder.begin(), porder.end(), [&](int x, int y) {
        return std::make_pair(lower_region(x), upper_region(x)) < std::make_pair(lower_region(y), upper_region(y));
    });
    for (int i : porder) {
        const int k = mesh->kind[i];
        if (k != GBEM_PANEL_NEUMANN) q_slot[i] = nu++;
        if (k == GBEM_PANEL_NEUMANN || k == GBEM_PANEL_INTERFACE) u_slot[i] = nu++;
    }
    // equations region by region, each region's rows from a multiple of 16
    // (gap rows: region -1, zero), and the slot range each region touches
    std::vector<int> row0(R, 0), nrows(R, 0), slo(R, INT32_MAX), shi(R, 0);
    int neq = 0;
    for (int a = 0; a < R; ++a) {
        while (eq_reg.size() % 16) {
            eq_reg.push_back(-1);
            eq_pan.push_back(0);
        }
        row0[a] = (int)eq_reg.size();
        for (int i = 0; i < n; ++i)
            if (mesh->region_plus[i] == a || mesh->region_minus[i] == a) {
                eq_reg.push_back(a);
                eq_pan.push_back(i);
                ++nrows[a];
                for (int sl : {q_slot[i], u_slot[i]})
                    if (sl >= 0) {
                        slo[a] = std::min(slo[a], sl);
                        shi[a] = std::max(shi[a], sl + 1);
                    }
            }
        neq += nrows[a];
    }
    while (eq_reg.size() % 16) {
        eq_reg.push_back(-1);
        eq_pan.push_back(0);
    }
    const int nrow = (int)eq_reg.size();
    if (neq != nu) {
        set_error("gbem_extract_dielectric: equations and unknowns do not match");
        return GBEM_EINVAL;
    }
    for (int k = 0; k < M; ++k) {
        bool any = false;
        for (int i = 0; i < n && !any; ++i) any = cond[i] == k;
        if (!any) {
            set_error("gbem_extract_dielectric: conductor " + std::to_string(k) + " has no panels");
            return GBEM_EINVAL;
        }
    }
    if (!ctx) {
        set_error("gbem_extract_dielectric: no context");
        return GBEM_EINVAL;
    }
    std::unique_lock<std::mutex> lk;
    if (!lane) {
        lk = std::unique_lock<std::mutex>(ctx->call_mu);
        HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
    }
    Workspace &ws = lane ? *lane->ws : ctx->ws;
    hipStream_t st = lane ? lane->st : ctx->stream;
    HIPCHK(ws.lo.ensure(sizeof(double) * 3 * n), "alloc mesh");
    HIPCHK(ws.hi.ensure(sizeof(double) * 3 * n), "alloc mesh");
    HIPCHK(ws.cond.ensure(sizeof(int32_t) * n), "alloc mesh");
    HIPCHK(hipMemcpyAsync(ws.lo.p, mesh->lo, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st), "H2D");
    HIPCHK(hipMemcpyAsync(ws.hi.p, mesh->hi, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st), "H2D");
    HIPCHK(hipMemcpyAsync(ws.cond.p, cond.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st), "H2D");
    // per-panel and per-equation tables and the conductor panels of each net
    // (CSR over nets) in one device block of int32
    Workspace::DlBufs &db = ws.dl;
    DevBuf &tab = db.tab, &epsb = db.epsb, &Q = db.Q, &Mb = db.M, &Mt = db.Mt, &Bb = db.B, &Bn = db.Bn, &Z = db.Z,
           &N = db.N, &X = db.X, &Rr = db.R, &D = db.D, &Cd = db.C, &nrm = db.nrm, &part = db.part;
    std::vector<int32_t> cp_ptr(M + 1, 0), cp_idx;
    for (int i = 0; i < n; ++i)
        if (cond[i] >= 0) ++cp_ptr[cond[i] + 1];
    for (int k = 0; k < M; ++k) cp_ptr[k + 1] += cp_ptr[k];
    cp_idx.resize(cp_ptr[M]);
    {
        std::vector<int32_t> fill(cp_ptr.begin(), cp_ptr.end() - 1);
        for (int i = 0; i < n; ++i)
            if (cond[i] >= 0) cp_idx[fill[cond[i]]++] = i;
    }
    const size_t ntab = (size_t)6 * n + 2 * (size_t)nrow + (M + 1) + cp_idx.size();
    HIPCHK(tab.ensure(sizeof(int32_t) * ntab), "alloc");
    std::vector<int32_t> htab(ntab);
    for (int i = 0; i < n; ++i) {
        htab[i] = mesh->kind[i];
        htab[n + i] = cond[i];
        htab[2 * n + i] = mesh->region_plus[i];
        htab[3 * n + i] = mesh->region_minus[i];
        htab[4 * n + i] = u_slot[i];
        htab[5 * n + i] = q_slot[i];
    }
    for (int r = 0; r < nrow; ++r) {
        htab[6 * (size_t)n + r] = eq_reg[r];
        htab[6 * (size_t)n + nrow + r] = eq_pan[r];
    }
    std::copy(cp_ptr.begin(), cp_ptr.end(), htab.begin() + 6 * (size_t)n + 2 * nrow);
    std::copy(cp_idx.begin(), cp_idx.end(), htab.begin() + 6 * (size_t)n + 2 * nrow + M + 1);
    HIPCHK(hipMemcpyAsync(tab.p, htab.data(), sizeof(int32_t) * ntab, hipMemcpyHostToDevice, st), "H2D");
    HIPCHK(epsb.ensure(sizeof(double) * R), "alloc");
    HIPCHK(hipMemcpyAsync(epsb.p, mesh->eps_r, sizeof(double) * R, hipMemcpyHostToDevice, st), "H2D");
    const int32_t *d_kind = tab.as<int32_t>(), *d_rp = d_kind + 2 * n, *d_rm = d_kind + 3 * n,
                  *d_us = d_kind + 4 * n, *d_qs = d_kind + 5 * n, *d_er = d_kind + 6 * (size_t)n,
                  *d_ep = d_er + nrow, *d_cpp = d_ep + nrow, *d_cpi = d_cpp + M + 1;
    int64_t nnz = 0;
    gbem_status s = dl_assemble(ws, n, M, o.near_eta, kDlNearEta, o.far_order, true, Q, &nnz, st);
    if (s != GBEM_OK) return s;
    const int64_t npadA = round_up(n, kPad), npad = round_up(std::max(nu, nrow), kPad);
    const auto t_asm = std::chrono::steady_clock::now();
    // the section 4.1 system M X = B (one column per main net), M and its
    // transpose zero-padded to order npad, B and -B to npad rows
    const size_t mat = (size_t)npad * npad * 8, vec = (size_t)npad * M * 8;
    HIPCHK(Mb.ensure(mat), "alloc M");
    HIPCHK(Mt.ensure(mat), "alloc M^T");
    HIPCHK(N.ensure(mat), "alloc N");
    for (DevBuf *v : {&Bb, &Bn, &Z, &X, &Rr, &D}) HIPCHK(v->ensure(vec), "alloc");
    HIPCHK(nrm.ensure(sizeof(double) * 2 * kMaxRhs), "alloc");
    HIPCHK(part.ensure((size_t)residual_splits((int)npad) * M * npad * 8), "alloc residual partials");
    for (DevBuf *v : {&Mb, &Mt, &N}) HIPCHK(hipMemsetAsync(v->p, 0, mat, st), "memset");
    for (DevBuf *v : {&Bb, &Bn, &Z, &X, &Rr, &D}) HIPCHK(hipMemsetAsync(v->p, 0, vec, st), "memset");
    HIPCHK(launch_dl_system(ws.pan.as<Panel>(), n, ws.A.as<double>(), npadA, Q.as<double>(), n, d_kind, d_rp, d_rm,
                            epsb.as<double>(), d_er, d_ep, d_us, d_qs, d_cpp, d_cpi, nrow, M, Mb.as<double>(),
                            Mt.as<double>(), npad, Bb.as<double>(), Bn.as<double>(), npad, st), "system");
    // normal equations (M^T M) X = M^T B on the FP64 Cholesky (the system is
    // not symmetric): M^T M on the factorisation's MFMA tiles (M^T is the
    // tile operand, rows = unknowns); the tall-skinny products through the
    // residual kernel, which forms B - A^T X:
    //   M^T B   = 0 - M^T (-B)      (A = M)
    //   B - M X                     (A = M^T)
    //   -M^T R  = 0 - M^T R         (A = M), subtracted from X
    // region by region: N = sum_a M_a^T M_a over region a's rows (K) and the
    // slot range its boundary touches (the rest of M_a is zero), accumulated
    // as -N on the subtracting tiles and negated once
    for (int a = 0; a < R; ++a) {
        if (nrows[a] == 0) continue;
        int64_t s0 = slo[a] / 128 * 128;
        const int64_t len = round_up(shi[a] - s0, 128);
        if (s0 + len > npad) s0 = npad - len;
        const int64_t K = round_up(nrows[a], 16);
        HIPCHK(launch_gram_f64(len, K, Mt.as<double>() + s0 + (int64_t)row0[a] * npad, npad,
                               N.as<double>() + s0 + s0 * npad, npad, true, st), "M^T M");
    }
    HIPCHK(launch_dl_negate(N.as<double>(), npad * npad, st), "M^T M");
    HIPCHK(launch_identity_pad(N.p, npad, nu, (int)npad, true, st), "pad");
    HIPCHK(launch_residual(Mb.as<double>(), npad, (int)npad, Bn.as<double>(), npad, Z.as<double>(), npad, M,
                           X.as<double>(), npad, part.as<double>(), st), "M^T B");
    HIPCHK(ws.Winv.ensure(chol_winv_bytes(GBEM_F64, npad)), "alloc W");
    HIPCHK(ws.Pw.ensure(chol_panel_bytes(GBEM_F64, npad)), "alloc panel");
    HIPCHK(ws.P16.ensure(std::max<size_t>(chol_panel16_bytes(GBEM_F64, npad), 64)), "alloc panel16");
    HIPCHK(hipMemsetAsync(ws.flags.p, 0, 64, st), "memset");
    hipStream_t la = st;
    if (!ws.lookahead_on_main) {
        HIPCHK(ws.ensure_side(), "side stream");
        la = ws.side;
    }
    HIPCHK(chol_factor(GBEM_F64, npad, N.p, npad, ws.Winv.p, ws.Pw.p, ws.P16.p, ws.flags.as<int32_t>() + 1, st, la,
                       ws.fev), "cholesky");
    int32_t ie[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(ie, ws.flags.as<int32_t>() + 1, 8, hipMemcpyDeviceToHost, st), "D2H");
    HIPCHK(hipStreamSynchronize(st), "sync");
    if (ie[1]) {
        set_error("Cholesky: a panel wait exceeded its poll limit");
        return GBEM_EDEVICE;
    }
    if (ie[0] != 0 && ie[0] <= nu) {
        set_error("gbem_extract_dielectric: the normal equations of the system are singular (check the mesh)");
        return GBEM_ENOTPD;
    }
    const auto t_fac = std::chrono::steady_clock::now();
    HIPCHK(ws.ensure_sync(npad, st), "alloc solve flags");
    HIPCHK(chol_solve_prep(GBEM_F64, npad, N.p, npad, ws.Winv.p, ws.sync, st), "solve prep");
    auto solve = [&](DevBuf &rhs) -> gbem_status {
        HIPCHK(hipMemsetAsync(ws.sync.err, 0, 4, st), "memset");
        HIPCHK(chol_solve(GBEM_F64, npad, N.p, npad, ws.Winv.p, M, rhs.as<double>(), npad, ws.sync, st), "solve");
        int32_t serr = 0;
        HIPCHK(hipMemcpyAsync(&serr, ws.sync.err, 4, hipMemcpyDeviceToHost, st), "D2H");
        HIPCHK(hipStreamSynchronize(st), "sync");
        if (serr) {
            set_error("triangular solve: a block wait exceeded its poll limit");
            return GBEM_EDEVICE;
        }
        return GBEM_OK;
    };
    if ((s = solve(X)) != GBEM_OK) return s;
    double bn[kMaxRhs], rn[kMaxRhs];
    HIPCHK(launch_col_norms(Bb.as<double>(), npad, (int)npad, M, nrm.as<double>(), st), "norms");
    HIPCHK(hipMemcpyAsync(bn, nrm.p, sizeof(double) * M, hipMemcpyDeviceToHost, st), "D2H");
    int iters = 0;
    double resid = 0.0;
    for (;; ++iters) {
        HIPCHK(launch_residual(Mt.as<double>(), npad, (int)npad, X.as<double>(), npad, Bb.as<double>(), npad, M,
                               Rr.as<double>(), npad, part.as<double>(), st), "residual");
        HIPCHK(launch_col_norms(Rr.as<double>(), npad, (int)npad, M, nrm.as<double>(), st), "norms");
        HIPCHK(hipMemcpyAsync(rn, nrm.p, sizeof(double) * M, hipMemcpyDeviceToHost, st), "D2H");
        HIPCHK(hipStreamSynchronize(st), "sync");
        double worst = 0.0;
        for (int k = 0; k < M; ++k) worst = std::max(worst, bn[k] > 0.0 ? sqrt(rn[k] / bn[k]) : sqrt(rn[k]));
        if (!(worst < INFINITY)) {
            set_error("gbem_extract_dielectric: the solution is not finite");
            return GBEM_ENOCONV;
        }
        resid = worst;
        if (worst <= 1e-13 || iters >= 6) break;
        HIPCHK(launch_residual(Mb.as<double>(), npad, (int)npad, Rr.as<double>(), npad, Z.as<double>(), npad, M,
                               D.as<double>(), npad, part.as<double>(), st), "M^T R");
        if ((s = solve(D)) != GBEM_OK) return s;
        HIPCHK(launch_dl_sub(X.as<double>(), npad, D.as<double>(), npad, (int)npad, M, st), "update");
    }
    HIPCHK(Cd.ensure(sizeof(double) * M * M), "alloc C");
    HIPCHK(launch_dl_charges(ws.pan.as<Panel>(), d_rp, d_rm, epsb.as<double>(), d_qs, d_cpp, d_cpi, X.as<double>(),
                             npad, M, kEps0 * mesh->length_unit_m, Cd.as<double>(), st), "charges");
    HIPCHK(hipMemcpyAsync(C_out, Cd.p, sizeof(double) * M * M, hipMemcpyDeviceToHost, st), "D2H");
    HIPCHK(hipStreamSynchronize(st), "sync");
    const auto t_end = std::chrono::steady_clock::now();
    if (rep) {
        gbem_report r{};
        auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
        r.t_assemble_ms = ms(t_start, t_asm);
        r.t_factor_ms = ms(t_asm, t_fac);
        r.t_solve_ms = ms(t_fac, t_end);
        r.t_total_ms = ms(t_start, t_end);
        r.residual = resid;
        r.refine_iters = iters;
        r.factor_used = GBEM_F64;
        r.n_near = nnz;
        r.n_panels = n;
        r.asym = asym_of(C_out, M);
        *rep = r;
    }
    return GBEM_OK;
}

extern "C" gbem_status gbem_extract_dielectric(gbem_ctx *ctx, const gbem_dmesh *mesh, const gbem_opts *opts,
                                               double *C_out, gbem_report *rep)
{
    return dielectric_run(ctx, nullptr, mesh, opts, C_out, rep);
}

// Column k of C from the mesh of main net k.  The meshes are built on the
// host first; the extractions then run on up to four lanes (host threads,
// each with a workspace and a stream of its own and the factorisation's
// look-ahead on that stream, so the context holds at most four streams
// besides its own), net k on lane k mod lanes.  Each column comes from one
// lane's kernels alone, so the result does not depend on the lane count.
extern "C" gbem_status gbem_extract_dielectric_partitioned(gbem_ctx *ctx, const gbem_dlayout *L,
                                                           const gbem_partition *rule, const gbem_opts *opts,
                                                           double *C_out, int32_t *panels_out, gbem_report *rep)
{
    if (!L || !rule || !C_out || L->n_conductors <= 0 || L->n_conductors > kMaxRhs || !L->eps_r) {
        set_error("gbem_extract_dielectric_partitioned: null argument or n_conductors outside 1..64");
        return GBEM_EINVAL;
    }
    const int M = L->n_conductors;
    std::vector<gbem_dmesh_buf> meshes(M);
    auto free_meshes = [&]() {
        for (auto &mb : meshes) gbem_dmesh_buf_free(&mb);
    };
    for (int k = 0; k < M; ++k) {
        const gbem_status s = gbem_mesh_dielectric_partition(L, k, rule, &meshes[k]);
        if (s != GBEM_OK) {
            free_meshes();
            return s;
        }
    }
    if (!ctx) {
        free_meshes();
        set_error("gbem_extract_dielectric_partitioned: no context");
        return GBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    const int lanes = std::min(M, 4);
    {
        hipError_t e = hipSetDevice(ctx->device);
        while (e == hipSuccess && (int)ctx->lane_ws.size() < lanes) {
            hipStream_t st = nullptr;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) break;
            ctx->lane_st.push_back(st);
            ctx->lane_ws.emplace_back(new Workspace());
            ctx->lane_ws.back()->lookahead_on_main = true;
        }
        if (e != hipSuccess) {
            free_meshes();
            set_error(std::string("gbem_extract_dielectric_partitioned: ") + hipGetErrorString(e));
            return GBEM_EDEVICE;
        }
    }
    std::vector<std::vector<double>> Ck(M, std::vector<double>((size_t)M * M));
    std::vector<gbem_report> reps(M);
    std::vector<gbem_status> stat(M, GBEM_OK);
    std::vector<std::string> errs(M);
    auto lane_main = [&](int l) {
        if (hipSetDevice(ctx->device) != hipSuccess) {
            for (int k = l; k < M; k += lanes) {
                stat[k] = GBEM_EDEVICE;
                errs[k] = "hipSetDevice failed on a lane";
            }
            return;
        }
        const Lane lane{ctx->lane_ws[l].get(), ctx->lane_st[l]};
        for (int k = l; k < M; k += lanes) {
            const gbem_dmesh_buf &mb = meshes[k];
            gbem_dmesh dm{};
            dm.n_panels = mb.n_panels;
            dm.n_conductors = M;
            dm.n_regions = L->n_layers;
            dm.lo = mb.lo;
            dm.hi = mb.hi;
            dm.kind = mb.kind;
            dm.conductor = mb.conductor;
            dm.region_plus = mb.region_plus;
            dm.region_minus = mb.region_minus;
            dm.eps_r = L->eps_r;
            dm.length_unit_m = L->length_unit_m;
            stat[k] = dielectric_run(ctx, &lane, &dm, opts, Ck[k].data(), &reps[k]);
            if (stat[k] != GBEM_OK) {
                errs[k] = gbem_last_error();   // the lane thread's message
                return;
            }
        }
    };
    std::vector<std::thread> th;
    for (int l = 1; l < lanes; ++l) th.emplace_back(lane_main, l);
    lane_main(0);
    for (auto &t : th) t.join();
    gbem_report tot{};
    for (int k = 0; k < M; ++k) {
        if (stat[k] != GBEM_OK) {
            free_meshes();
            set_error(errs[k]);
            return stat[k];
        }
        for (int n = 0; n < M; ++n) C_out[(size_t)n * M + k] = Ck[k][(size_t)n * M + k];
        if (panels_out) panels_out[k] = meshes[k].n_panels;
        const gbem_report &r = reps[k];
        tot.t_assemble_ms += r.t_assemble_ms;
        tot.t_factor_ms += r.t_factor_ms;
        tot.t_solve_ms += r.t_solve_ms;
        tot.t_total_ms += r.t_total_ms;
        tot.residual = std::max(tot.residual, r.residual);
        tot.refine_iters = std::max(tot.refine_iters, r.refine_iters);
        tot.n_near += r.n_near;
        tot.n_panels += r.n_panels;
        tot.factor_used = r.factor_used;
    }
    free_meshes();
    if (rep) {
        tot.asym = asym_of(C_out, M);
        *rep = tot;
    }
    return GBEM_OK;
}
