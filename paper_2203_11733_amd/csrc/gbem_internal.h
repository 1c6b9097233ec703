// Internal declarations shared by the HIP translation units of libgbem.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "gbem.h"

namespace gbem {

// Tile edge of the far-field assembly kernel and the padding unit of every
// device matrix: the order of A is padded to a multiple of kPad with an
// identity block, so the factorisation and solves need no edge cases.
constexpr int kFarTile = 64;
constexpr int kNB = 128;          // Cholesky block (diagonal block lives in LDS)
constexpr int kMaxPanelBlocks = 4;   // widest outer panel / kNB; chol_factor's info points at
                                     // 3 + 2 * kMaxPanelBlocks zeroed ints (pivot info, error word,
                                     // flags, ticket counter)
constexpr int kPad = 512;         // padding of the matrix order (one outer Cholesky panel)
constexpr int kMaxOrder = 8;      // largest Gauss order of the far rule
constexpr int kMaxRhs = 64;       // right-hand sides handled per solve pass
constexpr double kMinNearEta = 1e-6;   // smallest near threshold accepted

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Panel record in HBM: one 64-byte line per panel.
//   c[3]  centre, h1/h2 half-extents along the two in-plane axes (ascending
//   axis order), nrm normal axis, area, diam2 = |hi-lo|^2.
struct __attribute__((aligned(64))) Panel {
    double c[3];
    double h1, h2;
    double area;
    double diam2;
    int32_t nrm;
    int32_t cond;
};
static_assert(sizeof(Panel) == 64, "panel record must be one 64-byte line");

// Gauss-Legendre rule on [-1,1] passed by value to the far kernel.
// ww[a * p + b] = w_a w_b with w the Gauss weights halved (each direction
// sums to 1); xf/wwf are the same values rounded to FP32.
struct GaussRule {
    double x[kMaxOrder];
    double w[kMaxOrder];
    double ww[kMaxOrder * kMaxOrder];
    float xf[kMaxOrder];
    float wwf[kMaxOrder * kMaxOrder];
};

// Gauss rules of the semi-analytic near-pair route (halved weights): 10
// points per axis, 8 for pairs at least two sides apart.
constexpr int kNearOrder = 10, kNearOrderWide = 8;
struct NearRule {
    double x[kNearOrder];
    double w[kNearOrder];
    double x8[kNearOrderWide];
    double w8[kNearOrderWide];
};

// Event-based per-class kernel timing (opts.profile).  start() records an
// event on the stream; stop() records the closing event and the algorithmic
// work of the window; collect() sums the elapsed times after the final sync.
struct Prof {
    struct Rec {
        int cls;
        int a, b;
        double flops, bytes;
        int launches;
    };
    bool on = false;
    uint32_t mask = 0;             // classes timed (bit c = class c)
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;

    int event(hipStream_t s)
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            pool.push_back(e);
        }
        if (hipEventRecord(pool[used], s) != hipSuccess) return -1;
        return (int)used++;
    }
    int start(hipStream_t s, int cls) { return on && (mask >> cls & 1u) ? event(s) : -1; }
    void stop(int tok, int cls, double flops, double bytes, hipStream_t s, int launches = 1)
    {
        if (!on || tok < 0) return;
        int b = event(s);
        if (b >= 0) recs.push_back(Rec{cls, tok, b, flops, bytes, launches});
    }
    void reset()
    {
        used = 0;
        recs.clear();
    }
    void collect(gbem_report *rep)
    {
        if (!on || !rep) return;
        for (const Rec &r : recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pool[r.a], pool[r.b]) != hipSuccess) continue;
            rep->prof_ms[r.cls] += ms;
            rep->prof_launches[r.cls] += r.launches;
            rep->prof_flops[r.cls] += r.flops;
            rep->prof_bytes[r.cls] += r.bytes;
        }
    }
    ~Prof()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// ---- host helpers --------------------------------------------------------
void set_error(const std::string &msg);
// p-point Gauss-Legendre nodes (ascending) and halved weights on [-1, 1]
void gauss_legendre(int p, double *x, double *w_half);
void gauss_legendre_rule(int p, GaussRule *r);

// ---- kernel launchers (each returns hipSuccess or the launch error) ------
// panels.hip
hipError_t launch_build_panels(const double *lo, const double *hi, const int32_t *cond, int n,
                               int n_cond, Panel *pan, int32_t *bad, hipStream_t s);
hipError_t launch_rhs(const int32_t *cond, int n, int npad, int m, double *B, int64_t ldb,
                      hipStream_t s);
hipError_t launch_charge_partials(const double *X, int64_t ldx, const int32_t *cond, int n, int m,
                                  double *partial, int nchunks, hipStream_t s);
hipError_t launch_charge_finish(const double *partial, int nchunks, int m, double scale,
                                double *C, hipStream_t s);
hipError_t launch_gather(const double *A, int64_t lda, const int32_t *ii, const int32_t *jj, int64_t m,
                         double *out, hipStream_t s);
hipError_t launch_gather(const float *A, int64_t lda, const int32_t *ii, const int32_t *jj, int64_t m, float *out,
                         hipStream_t s);
hipError_t launch_identity_pad(void *A, int64_t lda, int n, int npad, bool f64, hipStream_t s);

// near.hip (compiled with -ffp-contract=off: the near/far test is bit-exact)
// mask: n * near_mask_words(n) words, written by near_count, read by near_fill
inline int64_t near_mask_words(int64_t n) { return (n + 63) / 64; }
hipError_t launch_near_count(const double *lo, const double *hi, int n, double eta2,
                             int64_t *cnt, uint64_t *mask, hipStream_t s);
hipError_t launch_exclusive_scan(const int64_t *cnt, int n, int64_t *row_ptr, hipStream_t s);
hipError_t launch_near_fill(const uint64_t *mask, int n, const int64_t *row_ptr, int32_t *row, int32_t *col,
                            hipStream_t s);

// near_eval.hip: closed-form Galerkin integrals of the near pairs.
// semi_buf: near_semi_bytes(nnz) bytes of scratch (queue of semi-analytic pairs)
// F, sc (optional, together): also F[i + j ldf] = (float)(sc_i a_ij sc_j) for
// the near pairs (j <= i), the scaled FP32 copy the mixed-precision factor uses
hipError_t launch_near_eval(const double *lo, const double *hi, const Panel *pan,
                            const int32_t *row, const int32_t *col, int64_t nnz, double *A,
                            int64_t lda, int32_t *semi_buf, hipStream_t s, float *F = nullptr,
                            int64_t ldf = 0, const double *sc = nullptr, bool upload_rule = true);
// the reductions' Gauss rules to constant memory (launch_near_eval does it
// itself unless upload_rule is false: inside a captured region)
hipError_t near_eval_upload_rule(hipStream_t s);
// sc[i] = a_ii^(-1/2) from the self integrals of the panels (the values the
// near pass writes on the diagonal), 1 for the padding rows [n, npad)
hipError_t launch_self_scale(const double *lo, const double *hi, const Panel *pan, int n, int npad, double *sc,
                             hipStream_t s);
inline size_t near_semi_bytes(int64_t nnz) { return (size_t)(64 + nnz) * sizeof(int32_t); }

// far.hip
// F, sc (optional, together): also the scaled FP32 lower triangle (see
// launch_near_eval); near entries are overwritten by the near pass
hipError_t launch_far(const Panel *pan, int n, int npad, int p, const GaussRule &rule,
                      int far_dtype, double *A, int64_t lda, hipStream_t s, float *F = nullptr,
                      int64_t ldf = 0, const double *sc = nullptr);

// tune.cpp: tile shapes of the factorisation per matrix order and factor
// dtype (the autotuner's cache, else built-in defaults); tuning_autoload
// reads the default cache once (GBEM_TUNE_FILE or tune_gfx950.json next to
// the library)
struct CholShape {
    int outer_width;    // columns per outer panel: 256 or 512
    int super_panels;   // outer panels per 16-bit trailing update: 2 or 4 (1 for FP32/FP64)
};
CholShape chol_shape(int dtype, int64_t npad);
void tuning_autoload();

// chol.hip
// side: second stream for the look-ahead panel factorisation; ev: event pool
hipError_t chol_factor(int dtype, int64_t npad, void *A, int64_t lda, void *Winv, void *panel,
                       void *panel16, int32_t *info, hipStream_t s, hipStream_t side,
                       std::vector<hipEvent_t> &ev, Prof *prof = nullptr);
// Synchronisation words of the persistent triangular solves (device arrays of
// npad/128 flags per direction, zeroed once when allocated).  err[0] is the
// error word (zeroed by the caller before a solve, read back after it);
// err[1], err[2] are the ticket counters of the forward and backward launches.
struct SolveSync {
    int32_t *flags_f = nullptr;
    int32_t *flags_b = nullptr;
    int32_t *err = nullptr;
    int32_t epoch = 0;
    uint32_t base_f = 0, base_b = 0;   // host copies of the two ticket counters
    // FP32 solves: published blocks (2 directions x npad x kMaxPub words) and
    // the products M_k, N_k, M2_k, N2_k (4 x npad x 128 floats) of the
    // factor prepared last
    uint64_t *pub = nullptr;
    float *sub = nullptr;
    const void *prep_of = nullptr;
    int64_t prep_npad = 0;
};
constexpr int kMaxPub = 64;
// solve.hip
hipError_t chol_solve(int dtype, int64_t npad, const void *L, int64_t lda, const void *Winv,
                      int m, double *B, int64_t ldb, SolveSync &sync, hipStream_t s,
                      Prof *prof = nullptr);
// M_k and N_k of a new FP32 factor (no-op for FP64); required before chol_solve
hipError_t chol_solve_prep(int dtype, int64_t npad, const void *L, int64_t lda, const void *Winv,
                           SolveSync &sync, hipStream_t s);
constexpr int kResMaxSplit = 16;
int residual_splits(int npad);
size_t chol_winv_bytes(int dtype, int64_t npad);
size_t chol_panel_bytes(int dtype, int64_t npad);
size_t chol_panel16_bytes(int dtype, int64_t npad);
// lower triangle of C = P P^T, or C -= P P^T with subtract (FP64 MFMA, the
// factorisation's trailing-update tiles): P is nrows x K column-major (nrows
// a multiple of 128, K of 16); the upper triangle of C's diagonal tiles keeps
// its old values
hipError_t launch_gram_f64(int64_t nrows, int64_t K, const double *P, int64_t ldp, double *C, int64_t ldc,
                           bool subtract, hipStream_t s);
// A = -A over n elements
hipError_t launch_dl_negate(double *A, int64_t n, hipStream_t s);
// W_k = inverse of the 128 x 128 diagonal blocks of an existing factor L
hipError_t chol_diag_inverses(int dtype, int64_t npad, const void *L, int64_t lda, void *Winv,
                              hipStream_t s);

// refine.hip: mixed-precision helpers; p[0..n) = v as a kernel (no memset
// node in a captured stream)
hipError_t launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t st);
// refine.hip: mixed-precision helpers
hipError_t launch_jacobi_scale(const double *A, int64_t lda, int npad, double *s, hipStream_t st);
hipError_t launch_scale_convert(const double *A, int64_t lda, const double *s, int npad,
                                float *F, int64_t ldf, hipStream_t st);
// partial: residual_splits(npad) * m * npad doubles
hipError_t launch_residual(const double *A, int64_t lda, int npad, const double *X, int64_t ldx,
                           const double *B, int64_t ldb, int m, double *R, int64_t ldr,
                           double *partial, hipStream_t st);
hipError_t launch_col_norms(const double *R, int64_t ldr, int npad, int m, double *norms,
                            hipStream_t st);
hipError_t launch_scale_rows(double *X, int64_t ldx, const double *s, int npad, int m,
                             hipStream_t st);
hipError_t launch_axpy_cols(double *X, int64_t ldx, const double *D, int64_t ldd, int npad, int m,
                            hipStream_t st);

// dielectric.hip: multi-dielectric case
// Q[i + k ldq] = double-layer integral of target panel i and source panel k
// (normal of k along + its axis), every pair: far rule, then the near pairs
// (row, col: the near list, col <= row) in both orders
hipError_t launch_double_layer(const Panel *pan, int n, const int32_t *row, const int32_t *col, int64_t nnz,
                               double *Q, int64_t ldq, hipStream_t s);
// system matrix M (nu x nu, zeroed by the caller) and its transpose Mt (both
// column-major), right-hand sides B and -B (nu x m_main) of the
// region-by-region equations; A: single-layer entries (normalised by the two
// areas), Q: double-layer integrals.  cp_ptr / cp_idx: the conductor panels
// of each net (CSR over nets, panel order)
hipError_t launch_dl_system(const Panel *pan, int n, const double *A, int64_t lda, const double *Q, int64_t ldq,
                            const int32_t *kind, const int32_t *rp, const int32_t *rm, const double *eps,
                            const int32_t *eq_reg, const int32_t *eq_pan, const int32_t *u_slot,
                            const int32_t *q_slot, const int32_t *cp_ptr, const int32_t *cp_idx, int nu, int m_main,
                            double *M, double *Mt, int64_t ldm, double *B, double *Bneg, int64_t ldb, hipStream_t s);
// C[k m_main + m] = scale * sum over the panels of conductor k of eps q |I|
hipError_t launch_dl_charges(const Panel *pan, const int32_t *rp, const int32_t *rm, const double *eps,
                             const int32_t *q_slot, const int32_t *cp_ptr, const int32_t *cp_idx, const double *X,
                             int64_t ldx, int m_main, double scale, double *C, hipStream_t s);
// X -= D (rows x m)
hipError_t launch_dl_sub(double *X, int64_t ldx, const double *D, int64_t ldd, int rows, int m, hipStream_t s);

}  // namespace gbem
