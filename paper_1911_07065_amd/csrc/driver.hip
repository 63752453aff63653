// C ABI of the device path: matrix handle, polynomial setup (Algorithm 4
// step 1), chain application (Algorithms 1 and 3), PP-GMRES(m) with FP64
// iterative refinement (Algorithm 4 step 2), stability check (section 3.5)
// and the adjoint helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ppgmres.h"
#include "host_core.h"
#include "kernels.h"
#include "poly.h"

using namespace ppg;

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            set_error(std::string("HIP error ") + hipGetErrorString(e_) + " in " + #expr);         \
            return PP_EDEVICE;                                                                     \
        }                                                                                          \
    } while (0)

#define PP_TRY(expr)                     \
    do {                                 \
        pp_status s_ = (expr);           \
        if (s_ < 0) return s_;           \
    } while (0)

namespace {

constexpr double kBreakdownTol = 1e-14;
constexpr int kMaxDegree = 4096;
// relative inner-cycle target of a reduced-precision cycle (the FP64 outer
// refinement recomputes the true residual after every cycle)
constexpr double kInnerEta[3] = {0.0, 1e-6, 1e-2};

template <typename T>
pp_status dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return PP_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return PP_ENOMEM;
    }
    return PP_OK;
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

inline hipStream_t S(void *s) { return (hipStream_t)s; }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Krylov workspace of one precision.
struct Workspace {
    int m = -1;          // columns - 1 of V
    long ldv = 0;
    void *V = nullptr;   // ldv x (m+1)
    void *P0 = nullptr, *P1 = nullptr, *T = nullptr, *D = nullptr, *ACC = nullptr;
};

struct pp_matrix_s {
    int n = 0, nnz = 0;
    const int32_t *rowptr = nullptr, *colind = nullptr;
    const double *val = nullptr;
    float *val32 = nullptr;
    int32_t *tiles = nullptr;
    int ntiles = 0;
    int xcd_remap = 1;
    std::vector<int32_t> h_rowptr;
    Workspace ws[3];
    // reductions and FP64 vectors
    int ldp = 0;
    double *partial = nullptr;  // dot_blocks(n) x ldp
    double *npart = nullptr;    // ceil(n/256)
    double *small = nullptr;    // h1 | h2 | H | inv | z   (5 * ldp)
    double *hpin = nullptr;     // pinned host mirror (2 * ldp)
    double *r64 = nullptr, *t64 = nullptr;
    int nblk_dot = 0, nblk_upd = 0;

    DevCSR dev() const {
        DevCSR d;
        d.n = n;
        d.nnz = nnz;
        d.rowptr = rowptr;
        d.colind = colind;
        d.val64 = val;
        d.val32 = val32;
        d.tiles = tiles;
        d.ntiles = ntiles;
        d.xcd_remap = xcd_remap;
        return d;
    }
    double *h1() { return small; }
    double *h2() { return small + ldp; }
    double *H() { return small + 2 * ldp; }
    double *inv() { return small + 3 * ldp; }
    double *z() { return small + 4 * ldp; }

    void release_ws(Workspace &w) {
        dev_free(w.V);
        dev_free(w.P0);  // P1, T, D and ACC live in P0's allocation
        w.P1 = w.T = w.D = w.ACC = nullptr;
        w.m = -1;
    }

    // Reduction buffers for up to `cols` Krylov columns.
    pp_status ensure_red(int cols) {
        if (cols + 2 <= ldp) return PP_OK;
        int want = std::max(cols + 2, 64);
        dev_free(partial);
        dev_free(small);
        if (hpin) (void)hipHostFree(hpin);
        hpin = nullptr;
        ldp = 0;
        PP_TRY(dev_alloc(&partial, (size_t)nblk_dot * want));
        PP_TRY(dev_alloc(&small, (size_t)5 * want));
        if (hipHostMalloc((void **)&hpin, sizeof(double) * 2 * want, hipHostMallocDefault) != hipSuccess) {
            hpin = nullptr;
            set_error("hipHostMalloc failed");
            return PP_ENOMEM;
        }
        ldp = want;
        return PP_OK;
    }

    pp_status ensure_ws(int prec, int m) {
        Workspace &w = ws[prec];
        PP_TRY(ensure_red(std::max(m, 1)));
        if (w.m >= m && w.P0) return PP_OK;
        release_ws(w);
        const size_t es = elem_size(prec);
        w.ldv = ((long)n + 63) / 64 * 64;
        const size_t vec = (size_t)w.ldv * es;
        char *p = nullptr;
        PP_TRY(dev_alloc(&p, vec * (size_t)(m + 1)));
        w.V = p;
        char *q = nullptr;
        PP_TRY(dev_alloc(&q, vec * 5));
        w.P0 = q;
        w.P1 = q + vec;
        w.T = q + 2 * vec;
        w.D = q + 3 * vec;
        w.ACC = q + 4 * vec;
        w.m = m;
        return PP_OK;
    }

    ~pp_matrix_s() {
        for (auto &w : ws) release_ws(w);
        dev_free(val32);
        dev_free(tiles);
        dev_free(partial);
        dev_free(npart);
        dev_free(small);
        dev_free(r64);
        if (hpin) (void)hipHostFree(hpin);
    }
};

namespace {

void *vcol(const Workspace &w, int prec, int j) { return (char *)w.V + (size_t)j * w.ldv * elem_size(prec); }

void *buf_ptr(int b, const void *in, void *out, const Workspace &w) {
    switch (b) {
        case B_IN:
            return (void *)in;
        case B_OUT:
            return out;
        case B_P0:
            return w.P0;
        case B_P1:
            return w.P1;
        case B_T:
            return w.T;
        default:
            return nullptr;
    }
}

pp_status run_program(pp_matrix A, const std::vector<Step> &prog, int prec, const void *in, void *out,
                      hipStream_t st) {
    const Workspace &w = A->ws[prec];
    const DevCSR d = A->dev();
    for (const Step &s : prog) {
        StepPtrs p;
        p.in = buf_ptr(s.in, in, out, w);
        p.aux = buf_ptr(s.aux, in, out, w);
        p.vfin = s.fin ? in : nullptr;
        p.out = buf_ptr(s.out, in, out, w);
        p.acc = buf_ptr(s.acc, in, out, w);
        p.acc_init = s.acc_init;
        p.spmv = s.spmv;
        p.a0 = s.a0;
        p.a1 = s.a1;
        p.a2 = s.a2;
        p.b0 = s.b0;
        p.b1 = s.b1;
        HIP_TRY(launch_chain_step(d, prec, p, st));
    }
    return PP_OK;
}

// One step of the SpMV alone: out = a0 * A in + a2 * aux
pp_status spmv_axpby(pp_matrix A, int prec, const void *in, double a0, const void *aux, double a2, void *out,
                     hipStream_t st) {
    StepPtrs p;
    p.in = in;
    p.aux = aux;
    p.vfin = nullptr;
    p.out = out;
    p.acc = nullptr;
    p.acc_init = 0;
    p.spmv = 1;
    p.a0 = a0;
    p.a1 = 0.0;
    p.a2 = a2;
    p.b0 = p.b1 = 0.0;
    HIP_TRY(launch_chain_step(A->dev(), prec, p, st));
    return PP_OK;
}

// Orthogonalise w = V[:, j+1] against V[:, 0..j] by classical Gram-Schmidt
// applied twice, normalise it, and leave the Hessenberg column
// (j+2 values) in A->hpin (host) after a stream synchronisation.
pp_status cgs2_step(pp_matrix A, int prec, const Workspace &ws, int j, hipStream_t st) {
    const int n = A->n;
    const int ncols = j + 1;
    void *w = vcol(ws, prec, j + 1);
    HIP_TRY(launch_dots(prec, n, ws.V, ws.ldv, ncols, w, A->partial, A->ldp, st));
    HIP_TRY(launch_reduce(A->nblk_dot, A->partial, A->ldp, ncols, A->h1(), A->H(), 1, st));
    HIP_TRY(launch_update(prec, n, ws.V, ws.ldv, ncols, A->h1(), w, nullptr, st));
    HIP_TRY(launch_dots(prec, n, ws.V, ws.ldv, ncols, w, A->partial, A->ldp, st));
    HIP_TRY(launch_reduce(A->nblk_dot, A->partial, A->ldp, ncols, A->h2(), A->H(), 2, st));
    HIP_TRY(launch_update(prec, n, ws.V, ws.ldv, ncols, A->h2(), w, A->npart, st));
    HIP_TRY(launch_reduce_norm(A->nblk_upd, A->npart, A->H() + ncols, A->inv(), st));
    HIP_TRY(launch_scale_cast(prec, prec, n, w, A->inv(), 0.0, w, st));
    HIP_TRY(hipMemcpyAsync(A->hpin, A->H(), sizeof(double) * (ncols + 1), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PP_OK;
}

// ||x|| of a device vector (synchronises); x is not modified.
pp_status dev_norm(pp_matrix A, int prec, const void *x, double *out, hipStream_t st) {
    HIP_TRY(launch_dots(prec, A->n, x, 0, 1, x, A->partial, A->ldp, st));
    HIP_TRY(launch_reduce(A->nblk_dot, A->partial, A->ldp, 1, A->h1(), nullptr, 0, st));
    HIP_TRY(hipMemcpyAsync(A->hpin, A->h1(), sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(A->hpin[0]);
    return PP_OK;
}

bool valid_prec(int p) { return p >= 0 && p <= 2; }

}  // namespace

extern "C" {

pp_status pp_matrix_create(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind, const double *val,
                           void *stream, pp_matrix *out) {
    if (!out || n <= 0 || nnz < 0 || n >= (1LL << 31) || nnz >= (1LL << 31) || !rowptr || (nnz > 0 && (!colind || !val))) {
        set_error("pp_matrix_create: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    auto *A = new (std::nothrow) pp_matrix_s();
    if (!A) return PP_ENOMEM;
    auto fail = [&](pp_status s) {
        delete A;
        return s;
    };
    A->n = (int)n;
    A->nnz = (int)nnz;
    A->rowptr = rowptr;
    A->colind = colind;
    A->val = val;
    A->h_rowptr.resize(n + 1);
    if (hipMemcpyAsync(A->h_rowptr.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("pp_matrix_create: cannot read rowptr");
        return fail(PP_EDEVICE);
    }
    const auto &rp = A->h_rowptr;
    if (rp[0] != 0 || rp[n] != nnz) {
        set_error("pp_matrix_create: rowptr[0] must be 0 and rowptr[n] must be nnz");
        return fail(PP_EINVAL);
    }
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) {
            set_error("pp_matrix_create: rowptr not non-decreasing");
            return fail(PP_EINVAL);
        }
    if (nnz > 0) {
        std::vector<int32_t> ci(nnz);
        if (hipMemcpyAsync(ci.data(), colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("pp_matrix_create: cannot read colind");
            return fail(PP_EDEVICE);
        }
        for (int64_t k = 0; k < nnz; ++k)
            if (ci[k] < 0 || ci[k] >= n) {
                set_error("pp_matrix_create: column index out of range");
                return fail(PP_EINVAL);
            }
    }
    // row tiles: <= kTileNnz stored entries and <= kTileRowsMax rows, or one long row
    std::vector<int32_t> tiles;
    tiles.push_back(0);
    int r = 0;
    while (r < n) {
        const int start = r;
        long nz = 0;
        while (r < n && r - start < kTileRowsMax) {
            const long rn = rp[r + 1] - rp[r];
            if (r > start && nz + rn > kTileNnz) break;
            nz += rn;
            ++r;
            if (rn > kTileNnz) break;
        }
        tiles.push_back(r);
    }
    A->ntiles = (int)tiles.size() - 1;
    A->nblk_dot = dot_blocks(A->n);
    A->nblk_upd = (A->n + 255) / 256;
    pp_status s;
    if ((s = dev_alloc(&A->tiles, tiles.size())) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->val32, (size_t)std::max<int64_t>(nnz, 1))) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->npart, (size_t)A->nblk_upd)) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->r64, (size_t)2 * A->n)) != PP_OK) return fail(s);
    A->t64 = A->r64 + A->n;
    if ((s = A->ensure_red(64)) != PP_OK) return fail(s);
    if (hipMemcpyAsync(A->tiles, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        launch_val_to_f32((int)nnz, val, A->val32, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        set_error("pp_matrix_create: device upload failed");
        return fail(PP_EDEVICE);
    }
    *out = A;
    return PP_OK;
}

pp_status pp_matrix_set_values(pp_matrix A, const double *val, void *stream) {
    if (!A || (!val && A->nnz > 0)) {
        set_error("pp_matrix_set_values: bad argument");
        return PP_EINVAL;
    }
    A->val = val;
    HIP_TRY(launch_val_to_f32(A->nnz, val, A->val32, S(stream)));
    return PP_OK;
}

void pp_matrix_destroy(pp_matrix A) { delete A; }

pp_status pp_matrix_transpose(pp_matrix A, int32_t *rowptr_t, int32_t *colind_t, int32_t *perm, void *stream) {
    if (!A || !rowptr_t || (A->nnz > 0 && (!colind_t || !perm))) {
        set_error("pp_matrix_transpose: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const int n = A->n, nnz = A->nnz;
    std::vector<int32_t> ci(nnz), rpt(n + 1, 0), cit(nnz), pm(nnz);
    if (nnz) HIP_TRY(hipMemcpyAsync(ci.data(), A->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int k = 0; k < nnz; ++k) rpt[ci[k] + 1]++;
    for (int i = 0; i < n; ++i) rpt[i + 1] += rpt[i];
    std::vector<int32_t> fillp(rpt.begin(), rpt.end() - 1);
    const auto &rp = A->h_rowptr;
    for (int r = 0; r < n; ++r)
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const int q = fillp[ci[k]]++;
            cit[q] = r;
            pm[q] = k;
        }
    HIP_TRY(hipMemcpyAsync(rowptr_t, rpt.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    if (nnz) {
        HIP_TRY(hipMemcpyAsync(colind_t, cit.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(perm, pm.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return PP_OK;
}

pp_status pp_gather(int64_t nnz, const double *in, const int32_t *perm, double *out, void *stream) {
    if (nnz < 0 || nnz >= (1LL << 31) || (nnz > 0 && (!in || !perm || !out))) {
        set_error("pp_gather: bad argument");
        return PP_EINVAL;
    }
    HIP_TRY(launch_gather((int)nnz, in, perm, out, S(stream)));
    return PP_OK;
}

pp_status pp_adjoint_values(pp_matrix A, const double *lam, const double *x, double *dval, void *stream) {
    if (!A || !lam || !x || (A->nnz > 0 && !dval)) {
        set_error("pp_adjoint_values: bad argument");
        return PP_EINVAL;
    }
    HIP_TRY(launch_adjoint_values(A->dev(), lam, x, dval, S(stream)));
    return PP_OK;
}

pp_status pp_gmres_setup(pp_matrix A, const double *v0, int d, int add_roots, void *stream, pp_poly *out,
                         pp_setup_info *info) {
    if (!A || !v0 || !out || d < 1 || d > A->n || d > kMaxDegree) {
        set_error("pp_gmres_setup: bad argument (need 1 <= d <= min(n, 4096))");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    PP_TRY(A->ensure_ws(0, d));
    PP_TRY(A->ensure_red(d + 1));
    const Workspace &ws = A->ws[0];
    const int n = A->n;
    // V[:,0] = v0 / ||v0||
    void *v0c = vcol(ws, 0, 0);
    HIP_TRY(hipMemcpyAsync(v0c, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_update(0, n, ws.V, ws.ldv, 0, A->h1(), v0c, A->npart, st));
    HIP_TRY(launch_reduce_norm(A->nblk_upd, A->npart, A->H(), A->inv(), st));
    HIP_TRY(launch_scale_cast(0, 0, n, v0c, A->inv(), 0.0, v0c, st));
    HIP_TRY(hipMemcpyAsync(A->hpin, A->H(), sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!(A->hpin[0] > 0.0) || !std::isfinite(A->hpin[0])) {
        set_error("pp_gmres_setup: start vector is zero or not finite");
        return PP_EINVAL;
    }
    std::vector<double> Hbar((size_t)(d + 1) * d, 0.0);
    const int ld = d + 1;
    int k = d;
    bool brk = false;
    double fro2 = 0.0;
    int64_t dots = 1;
    for (int j = 0; j < d; ++j) {
        PP_TRY(spmv_axpby(A, 0, vcol(ws, 0, j), 1.0, nullptr, 0.0, vcol(ws, 0, j + 1), st));
        PP_TRY(cgs2_step(A, 0, ws, j, st));
        dots += 2 * (j + 1) + 1;
        for (int i = 0; i <= j + 1; ++i) {
            const double h = A->hpin[i];
            if (!std::isfinite(h)) {
                set_error("pp_gmres_setup: non-finite Hessenberg entry");
                return PP_EINVAL;
            }
            Hbar[(size_t)i + (size_t)j * ld] = h;
            fro2 += h * h;
        }
        if (Hbar[(size_t)(j + 1) + (size_t)j * ld] <= kBreakdownTol * std::sqrt(fro2)) {
            k = j + 1;
            brk = true;
            break;
        }
    }
    // repack to (k+1) x k
    std::vector<double> hk((size_t)(k + 1) * k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i <= k; ++i) hk[(size_t)i + (size_t)j * (k + 1)] = Hbar[(size_t)i + (size_t)j * ld];
    std::vector<double> re(k), im(k);
    int hs = harmonic_ritz(k, hk.data(), brk, re.data(), im.data());
    if (hs != PP_OK) {
        if (hs == PP_ESINGULAR) set_error("pp_gmres_setup: singular H_dd or zero harmonic Ritz value");
        return (pp_status)hs;
    }
    auto *p = new (std::nothrow) pp_poly_s();
    if (!p) return PP_ENOMEM;
    int ps = plan_roots(k, re.data(), im.data(), add_roots != 0, p->plan);
    if (ps != PP_OK) {
        delete p;
        return (pp_status)ps;
    }
    p->theta_re = re;
    p->theta_im = im;
    p->breakdown = brk ? 1 : 0;
    p->finalize();
    *out = p;
    if (info) {
        info->d = k;
        info->d_eff = p->plan.d_eff;
        info->n_added = p->plan.n_added;
        info->breakdown = brk ? 1 : 0;
        info->mvps = k;
        info->dots = dots;
        info->t_setup_s = now_s() - t0;
    }
    return (brk && k < d) ? PP_BREAKDOWN : PP_OK;
}

pp_status pp_apply(pp_poly p, pp_matrix A, int kind, int prec, const void *v, void *y, void *stream) {
    if (!p || !A || !v || !y || v == y || !valid_prec(prec) || kind < 0 || kind > 2) {
        set_error("pp_apply: bad argument");
        return PP_EINVAL;
    }
    PP_TRY(A->ensure_ws(prec, 0));
    const auto &prog = kind == PP_APPLY_P ? p->prog_p : (kind == PP_APPLY_PHI ? p->prog_phi : p->prog_pi);
    return run_program(A, prog, prec, v, y, S(stream));
}

pp_status pp_stability_check(pp_poly p, pp_matrix A, const double *b, void *stream, double *stch) {
    if (!p || !A || !b || !stch) {
        set_error("pp_stability_check: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    PP_TRY(A->ensure_ws(0, 0));
    const Workspace &ws = A->ws[0];
    // r1 = b - A p(A) b  (into ws.ACC); r2 = pi(A) b (into r64); ||r1 - r2||
    PP_TRY(run_program(A, p->prog_p, 0, b, ws.D, st));
    PP_TRY(spmv_axpby(A, 0, ws.D, -1.0, b, 1.0, ws.ACC, st));
    PP_TRY(run_program(A, p->prog_pi, 0, b, A->r64, st));
    HIP_TRY(hipStreamSynchronize(st));
    A->hpin[A->ldp] = 1.0;
    HIP_TRY(hipMemcpyAsync(A->h1(), A->hpin + A->ldp, sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_update(0, A->n, A->r64, A->n, 1, A->h1(), ws.ACC, A->npart, st));
    HIP_TRY(launch_reduce_norm(A->nblk_upd, A->npart, A->H(), A->inv(), st));
    HIP_TRY(hipMemcpyAsync(A->hpin, A->H(), sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *stch = A->hpin[0];
    return PP_OK;
}

pp_status pp_solve(pp_poly p, pp_matrix A, const double *b, double *x, const pp_solve_opts *opts, void *stream,
                   pp_info *info) {
    if (!p || !A || !b || !x || !opts || opts->m < 1 || opts->max_cycles < 0 || !(opts->tol > 0.0) ||
        !valid_prec(opts->inner)) {
        set_error("pp_solve: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    const int n = A->n;
    const int m = opts->m;
    PP_TRY(A->ensure_ws(0, m));
    if (opts->inner != PP_F64) PP_TRY(A->ensure_ws(opts->inner, m));
    PP_TRY(A->ensure_red(m + 1));
    pp_info inf;
    std::memset(&inf, 0, sizeof(inf));
    inf.relres_shortcut = NAN;
    double bnorm = 0.0;
    PP_TRY(dev_norm(A, 0, b, &bnorm, st));
    HIP_TRY(launch_fill(n, 0.0, x, st));
    inf.dots += 1;
    if (bnorm == 0.0) {
        HIP_TRY(hipStreamSynchronize(st));
        inf.status = PP_OK;
        inf.relres = 0.0;
        inf.t_solve_s = now_s() - t0;
        if (info) *info = inf;
        return PP_OK;
    }
    if (!std::isfinite(bnorm)) {
        set_error("pp_solve: right-hand side not finite");
        return PP_EINVAL;
    }
    // r = b
    HIP_TRY(hipMemcpyAsync(A->r64, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    double beta = bnorm;
    int prec = opts->inner;
    std::vector<double> hist;
    GivensLS ls;
    std::vector<double> zh(m + 1);
    const int dphi = p->plan.d_eff;
    const int64_t mv_phi = dphi, mv_p = dphi - 1;
    pp_status status = PP_OK;
    for (;;) {
        const double relres = beta / bnorm;
        hist.push_back(relres);
        inf.relres = relres;
        if (relres <= opts->tol) {
            status = PP_OK;
            break;
        }
        if (inf.cycles >= opts->max_cycles) {
            status = PP_NOCONV;
            break;
        }
        const int sc = opts->stall_cycles;
        if (sc > 0 && (int)hist.size() > sc && hist.back() > 0.99 * hist[hist.size() - 1 - sc]) {
            status = PP_NOCONV;
            break;
        }
        if (!std::isfinite(beta)) {
            status = PP_NOCONV;
            set_error("pp_solve: residual not finite");
            break;
        }
        inf.cycles++;
        if (prec == PP_F64) inf.fp64_cycles++;
        const Workspace &ws = A->ws[prec];
        // V[:,0] = r / beta in the cycle's precision
        HIP_TRY(launch_scale_cast(0, prec, n, A->r64, nullptr, 1.0 / beta, vcol(ws, prec, 0), st));
        ls.reset(m, beta);
        const double target = std::max(opts->tol * bnorm, kInnerEta[prec] * beta);
        double fro2 = 0.0;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            PP_TRY(run_program(A, p->prog_phi, prec, vcol(ws, prec, j), vcol(ws, prec, j + 1), st));
            PP_TRY(cgs2_step(A, prec, ws, j, st));
            inf.mvps += mv_phi;
            inf.dots += 2 * (j + 1) + 1;
            inf.vops += 4 * (j + 1) + 2 + (int64_t)p->prog_phi.size();
            inf.iters++;
            bool finite = true;
            for (int i = 0; i <= j + 1; ++i) {
                finite = finite && std::isfinite(A->hpin[i]);
                fro2 += A->hpin[i] * A->hpin[i];
            }
            if (!finite) {
                set_error("pp_solve: non-finite Hessenberg entry");
                k = j;  // drop this column
                break;
            }
            const double shortcut = ls.add_column(A->hpin);
            k = j + 1;
            inf.relres_shortcut = shortcut / bnorm;
            const bool lucky = A->hpin[j + 1] <= kBreakdownTol * std::sqrt(fro2);
            if (lucky || shortcut <= target) break;
        }
        if (k > 0) {
            ls.solve(zh.data());
            // stage through pinned memory (the stream is idle here: cgs2_step synchronised)
            std::memcpy(A->hpin + A->ldp, zh.data(), sizeof(double) * k);
            HIP_TRY(hipMemcpyAsync(A->z(), A->hpin + A->ldp, sizeof(double) * k, hipMemcpyHostToDevice, st));
            // dy = V_k z (z solves min ||beta e1 - Hbar z||, so it carries beta);
            // dx = p(A) dy ; x += dx in FP64
            HIP_TRY(launch_combine(prec, n, ws.V, ws.ldv, k, A->z(), ws.D, st));
            PP_TRY(run_program(A, p->prog_p, prec, ws.D, ws.ACC, st));
            HIP_TRY(launch_axpy_x(prec, n, 1.0, ws.ACC, x, st));
            inf.mvps += mv_p;
            inf.vops += k + (int64_t)p->prog_p.size() * 2 + 1;
        }
        // true residual in FP64: r = b - A x
        PP_TRY(spmv_axpby(A, 0, x, -1.0, b, 1.0, A->r64, st));
        inf.mvps += 1;
        double beta_new = 0.0;
        PP_TRY(dev_norm(A, 0, A->r64, &beta_new, st));
        inf.dots += 1;
        inf.vops += 2;
        if (prec != PP_F64 && !(beta_new <= 0.5 * beta)) prec = PP_F64;  // refinement stalls: finish in FP64
        beta = beta_new;
    }
    inf.status = status;
    inf.t_solve_s = now_s() - t0;
    if (info) *info = inf;
    return status;
}

}  // extern "C"
