// C ABI of the device path: matrix handle, polynomial setup (Algorithm 4
// step 1), chain application (Algorithms 1 and 3), PP-GMRES(m) with FP64
// iterative refinement (Algorithm 4 step 2), stability check (section 3.5)
// and the adjoint helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/ppgmres.h"
#include "host_core.h"
#include "kernels.h"
#include "poly.h"
#include "common.h"

using namespace ppg;

namespace {

constexpr double kBreakdownTol = 1e-14;
constexpr int kMaxDegree = 4096;
// relative inner-cycle target of a reduced-precision cycle (the FP64 outer
// refinement recomputes the true residual after every cycle)
constexpr double kInnerEta[3] = {0.0, 1e-5, 1e-2};
// The host's round trip between an Arnoldi step's column and the next
// launches (what a queued-ahead phi(A) hides), in microseconds; and the time
// per chain launch assumed when the precision was not tuned.
constexpr double kLookaheadGapUs = 15.0;
constexpr double kLaunchGuessUs = 5.0;

}  // namespace

// Krylov workspace of one precision.
struct Workspace {
    int m = -1;          // columns - 1 of V
    long ldv = 0;
    void *V = nullptr;   // ldv x (m+1)
    void *P0 = nullptr, *P1 = nullptr, *T = nullptr, *D = nullptr, *ACC = nullptr;
    void *X = nullptr;  // 5 more vectors for composite polynomials (allocated on first use)
};

struct pp_matrix_s {
    int n = 0, nnz = 0;
    const int32_t *rowptr = nullptr, *colind = nullptr;
    const double *val = nullptr;
    float *val32 = nullptr;
    int4 *tile8 = nullptr, *tile16 = nullptr, *tileP = nullptr;
    int ntile8 = 0, ntile16 = 0, ntileP = 0;
    int4 *tileB8[3] = {nullptr, nullptr, nullptr}, *tileB16[3] = {nullptr, nullptr, nullptr};
    // sliced-ELL copy
    int32_t *sptr = nullptr, *scol = nullptr, *sperm = nullptr;
    int16_t *sdel = nullptr;
    // diagonal-format copy (few diagonals only): values diagonal-major, and
    // for each slot the CSR entry it holds (-1: zero padding)
    std::vector<int> h_doff;
    double *dval64 = nullptr;
    float *dval32 = nullptr;
    int32_t *dperm = nullptr;
    // value-coded diagonal copy (few distinct values; dropped when the values change)
    uint8_t *dcode = nullptr;
    double *dtab64 = nullptr;
    float *dtab32 = nullptr;
    int ntab = 0;
    // for new values with the same codes: each entry's code, one entry per
    // code, each pattern's code tuple, and the check's flag
    uint8_t *ecode = nullptr;
    int32_t *crep = nullptr;
    uint8_t *pcodes = nullptr;
    int *rflag = nullptr;
    bool recoded = false;  // the codes were rebuilt once from new values
    // block-Jacobi right preconditioner of a handle made for B = A M^{-1}:
    // pp_solve returns x = M^{-1} x~ (blocks of rbs rows, stride rbs)
    int rbs = 0;
    double *rminv = nullptr;
    // box geometry of a 5- or 7-point stencil matrix (box_nd == 0: none) and,
    // per precision, whether chains run two real-root steps per launch and
    // the tuned time of one such launch
    int box[3] = {0, 0, 0};
    int box_nd = 0;
    int box_pint = -1;  // constant-coefficient box stencil: the interior row's pattern (-1: not one)
    int fuse[3] = {0, 0, 0};
    double pair_us[3] = {0, 0, 0};
    // per precision: chains run up to march[prec] consecutive steps per
    // launch of the marching kernel (0: off), with chunks of march_cz planes;
    // march_us[prec][g] is the tuned time of one g-step launch (0: not timed)
    int march[3] = {0, 0, 0};
    int march_all[3] = {0, 0, 0};  // set by hand: every group of >= 2 steps marches
    int march_cz[3][kMarchMax + 1] = {};
    int march_depth[3][kMarchMax + 1] = {};  // planes of loads in flight (1..3)
    double march_us[3][kMarchMax + 1] = {};
    // per precision: two-step launches run the whole-line tile kernel
    // instead of marching planes (constant-coefficient 7-point stencils)
    int march_tile[3] = {0, 0, 0};
    int tile_remap[3] = {1, 1, 1};
    // per precision: two-step pairs (p chains' steps with the accumulator)
    // run the whole-line tile kernel instead of the cube-tile pair kernel
    int pair_tile[3] = {0, 0, 0};
    int pair_remap[3] = {1, 1, 1};
    // column-banded CSR copies (matrices whose entries lie far from the
    // diagonal): c = 0 two bands, c = 1 four; bperm maps entries to CSR
    int32_t *brow[2] = {nullptr, nullptr}, *bcol[2] = {nullptr, nullptr}, *bperm[2] = {nullptr, nullptr};
    double *bval64[2] = {nullptr, nullptr};
    float *bval32[2] = {nullptr, nullptr};
    int4 *btile[2] = {nullptr, nullptr};
    int btoff[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    int bandK[2] = {0, 0};
    long bnnz[2] = {0, 0};
    double *bpart = nullptr;
    // column-sorted tiles (cs_nb == 0: none); cs_perm / cs_dperm map tile
    // entries and held-apart diagonal entries to CSR positions
    uint32_t *cs_code = nullptr;
    int32_t *cs_perm = nullptr, *cs_toff = nullptr, *cs_dperm = nullptr;
    uint16_t *cs_tptr = nullptr;
    double *cs_val64 = nullptr, *cs_dg64 = nullptr, *cs_part = nullptr;
    float *cs_val32 = nullptr, *cs_dg32 = nullptr;
    int cs_nb = 0, cs_sb = 0, cs_W = 0, cs_maxe = 0;
    long cs_nnz = 0;
    // pattern-coded diagonal copy (few distinct rows; dropped with the value codes)
    uint32_t *pcode = nullptr;
    uint8_t *pbyte = nullptr;
    double *ptab64 = nullptr;
    float *ptab32 = nullptr;
    int npat = 0;
    // right scaling A diag(s) (composition with a diagonal preconditioner):
    // the chains, the setup and the residual use the scaled values val_own;
    // pp_solve returns x = diag(s) x~
    int scale_mode = 0;                // 0 none, 1 Jacobi (s = 1/diag of the values), 2 the caller's s
    const double *user_val = nullptr;  // the caller's unscaled values
    double *val_own = nullptr;         // scaled values (nnz)
    double *scale = nullptr;           // s (n)
    double *sval64 = nullptr;
    float *sval32 = nullptr;
    int nslices = 0;
    long npad = 0;
    int ntileB8[3] = {0, 0, 0}, ntileB16[3] = {0, 0, 0};
    int variant[3] = {CV_TILE8, CV_TILE8, CV_TILE8};  // single-launch variant
    int remap[3] = {1, 1, 1};
    int persist[3] = {0, 0, 0};     // chains of >= 2 steps in one cooperative launch
    int premap[3] = {1, 1, 1};
    int tuned[3] = {0, 0, 0};
    double tuned_us[3] = {0, 0, 0};
    // persistent kernel state
    int pgrid = 0;
    int tune_persist = 0;
    unsigned long long *bar = nullptr;  // barrier counter (device)
    unsigned long long bar_host = 0;    // its value after the last launch
    int *err = nullptr;                 // barrier timeout flag (device)
    int *errpin = nullptr;              // pinned mirror
    bool persist_ran = false;           // a persistent launch happened (the flag can be set)
    PStep *tune_steps = nullptr;        // 8 alternating sparse products
    std::map<std::pair<unsigned long long, int>, PStep *> progs;  // (poly id, kind) -> device table
    std::vector<int32_t> h_rowptr;
    Workspace ws[3];
    // reductions and FP64 vectors
    int ldp = 0;
    double *partial = nullptr;  // max(dot_blocks, update_dots_blocks) x ldp
    double *npart = nullptr;    // ceil(n/256)
    double *small = nullptr;    // h1 | h2 | H | inv | z   (5 * ldp)
    double *hpin = nullptr;     // pinned host mirror (2 * ldp)
    double *r64 = nullptr, *t64 = nullptr;
    int nblk_dot = 0, nblk_upd = 0, nblk_ud = 0;

    DevCSR dev() const {
        DevCSR d;
        d.n = n;
        d.nnz = nnz;
        d.rowptr = rowptr;
        d.colind = colind;
        d.val64 = val;
        d.val32 = val32;
        d.tile8 = tile8;
        d.ntile8 = ntile8;
        d.tile16 = tile16;
        d.ntile16 = ntile16;
        d.tileP = tileP;
        d.ntileP = ntileP;
        d.sptr = sptr;
        d.scol = scol;
        d.sdel = sdel;
        d.sval64 = sval64;
        d.sval32 = sval32;
        d.nslices = nslices;
        d.doff.nd = (int)h_doff.size();
        for (int k = 0; k < kMaxDiag; ++k) d.doff.off[k] = k < d.doff.nd ? h_doff[k] : 0;
        d.dval64 = dval64;
        d.dval32 = dval32;
        d.dcode = dcode;
        d.dtab64 = dtab64;
        d.dtab32 = dtab32;
        d.ntab = ntab;
        for (int c = 0; c < 2; ++c) {
            d.brow[c] = brow[c];
            d.bcol[c] = bcol[c];
            d.bval64[c] = bval64[c];
            d.bval32[c] = bval32[c];
            d.btile[c] = btile[c];
            for (int k = 0; k < 5; ++k) d.btoff[c][k] = btoff[c][k];
            d.bandK[c] = bandK[c];
        }
        d.bpart = bpart;
        d.cs_code = cs_code;
        d.cs_val64 = cs_val64;
        d.cs_val32 = cs_val32;
        d.cs_toff = cs_toff;
        d.cs_tptr = cs_tptr;
        d.cs_dg64 = cs_dperm ? cs_dg64 : nullptr;
        d.cs_dg32 = cs_dperm ? cs_dg32 : nullptr;
        d.cs_part = cs_part;
        d.cs_nb = cs_nb;
        d.cs_sb = cs_sb;
        d.cs_W = cs_W;
        d.cs_maxe = cs_maxe;
        d.pcode = pcode;
        d.pbyte = pbyte;
        d.ptab64 = ptab64;
        d.ptab32 = ptab32;
        d.npat = npat;
        for (int k = 0; k < 3; ++k) d.box[k] = box[k];
        d.box_nd = box_nd;
        d.box_pint = box_nd && pbyte ? box_pint : -1;
        for (int p = 0; p < 3; ++p) {
            d.tileB8[p] = tileB8[p];
            d.ntileB8[p] = ntileB8[p];
            d.tileB16[p] = tileB16[p];
            d.ntileB16[p] = ntileB16[p];
        }
        for (int p = 0; p < 3; ++p) {
            d.variant[p] = variant[p];
            d.remap[p] = remap[p];
        }
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
        dev_free(w.X);
        w.P1 = w.T = w.D = w.ACC = nullptr;
        w.m = -1;
    }

    // The 5 extra vectors of a precision (after ensure_ws).
    pp_status ensure_extra(int prec) {
        Workspace &w = ws[prec];
        if (w.X) return PP_OK;
        char *q = nullptr;
        PP_TRY(dev_alloc(&q, (size_t)w.ldv * elem_size(prec) * 5));
        w.X = q;
        return PP_OK;
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
        PP_TRY(dev_alloc(&partial, (size_t)std::max(nblk_dot, nblk_ud) * want));
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
        dev_free(tile8);
        dev_free(tile16);
        dev_free(tileP);
        dev_free(sptr);
        dev_free(scol);
        dev_free(sperm);
        dev_free(sdel);
        dev_free(dval64);
        dev_free(dval32);
        dev_free(dperm);
        dev_free(dcode);
        dev_free(dtab64);
        dev_free(dtab32);
        dev_free(ecode);
        dev_free(crep);
        dev_free(pcodes);
        dev_free(rflag);
        dev_free(rminv);
        dev_free(pcode);
        dev_free(pbyte);
        dev_free(ptab64);
        dev_free(ptab32);
        for (int c = 0; c < 2; ++c) {
            dev_free(brow[c]);
            dev_free(bcol[c]);
            dev_free(bperm[c]);
            dev_free(bval64[c]);
            dev_free(bval32[c]);
            dev_free(btile[c]);
        }
        dev_free(bpart);
        dev_free(cs_code);
        dev_free(cs_perm);
        dev_free(cs_toff);
        dev_free(cs_dperm);
        dev_free(cs_tptr);
        dev_free(cs_val64);
        dev_free(cs_val32);
        dev_free(cs_dg64);
        dev_free(cs_dg32);
        dev_free(cs_part);
        dev_free(val_own);
        dev_free(scale);
        dev_free(sval64);
        dev_free(sval32);
        for (int p = 0; p < 3; ++p) {
            dev_free(tileB8[p]);
            dev_free(tileB16[p]);
        }
        dev_free(bar);
        dev_free(err);
        dev_free(tune_steps);
        for (auto &kv : progs) dev_free(kv.second);
        if (errpin) (void)hipHostFree(errpin);
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

// Queue the copy of the barrier flag to the host, if a persistent launch
// ever ran on this handle (no other kernel sets it).
hipError_t copy_barrier_flag(pp_matrix A, hipStream_t st) {
    if (!A->persist_ran) return hipSuccess;
    return hipMemcpyAsync(A->errpin, A->err, sizeof(int), hipMemcpyDeviceToHost, st);
}

pp_status check_barrier_flag(pp_matrix A) {
    if (A->errpin && *A->errpin) {
        set_error("persistent chain: grid barrier timed out");
        return PP_EDEVICE;
    }
    return PP_OK;
}

PStep to_pstep(const Step &s) {
    PStep p;
    p.spmv = s.spmv;
    p.in = s.in;
    p.aux = s.aux;
    p.out = s.out;
    p.acc = s.acc;
    p.acc_init = s.acc_init;
    p.fin = s.fin;
    p.pad = 0;
    p.a0 = s.a0;
    p.a1 = s.a1;
    p.a2 = s.a2;
    p.b0 = s.b0;
    p.b1 = s.b1;
    return p;
}

pp_status upload_steps(const std::vector<PStep> &h, PStep **out, hipStream_t st) {
    PP_TRY(dev_alloc(out, h.size()));
    HIP_TRY(hipMemcpyAsync(*out, h.data(), sizeof(PStep) * h.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PP_OK;
}

pp_status launch_persist(pp_matrix A, int prec, const PStep *steps, int nsteps, const void *in, void *out, int remap,
                         hipStream_t st) {
    const Workspace &w = A->ws[prec];
    void *bufs[5] = {(void *)in, out, w.P0, w.P1, w.T};
    A->persist_ran = true;
    HIP_TRY(launch_chain_persist(A->dev(), prec, bufs, steps, nsteps, A->bar, A->bar_host, A->err, A->pgrid, remap,
                                 st));
    A->bar_host += (unsigned long long)(nsteps - 1) * (unsigned long long)A->pgrid;
    return PP_OK;
}

// Autotuner: per sparse product, time every single-launch chain variant
// (with and without the XCD-aware workgroup order) on 5 back-to-back
// launches, and the persistent kernel on an 8-step program; keep the
// fastest single-launch variant and use the persistent kernel for chains
// if it beats it.
// Tile plan with a whole number of occupancy rounds of equal tiles: every
// co-resident workgroup slot gets the same number of tiles of the same
// size, so the last round is not a partial one.
pp_status build_round_plan(pp_matrix A, int prec, int ept, int4 **dst, int *ndst, hipStream_t st) {
    if (*dst) return PP_OK;
    int slots = 0;
    HIP_TRY(tile_slots(prec, ept, &slots));
    if (slots <= 0) return PP_OK;
    const long cap_max = 256L * ept - 4, rows_max = 256L * (ept / 8);
    const long rounds = std::max<long>(1, ((long)A->nnz + slots * cap_max - 1) / (slots * cap_max));
    const long cap = std::max<long>(1, ((long)A->nnz + slots * rounds - 1) / (slots * rounds));
    std::vector<int4> t;
    build_tiles(A->h_rowptr.data(), A->n, (int)rows_max, (int)std::min(cap, cap_max), t);
    PP_TRY(dev_alloc(dst, t.size()));
    HIP_TRY(hipMemcpyAsync(*dst, t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    *ndst = (int)t.size();
    return PP_OK;
}

pp_status tune_chain(pp_matrix A, int prec, hipStream_t st) {
    PP_TRY(A->ensure_ws(prec, 0));
    PP_TRY(build_round_plan(A, prec, 8, &A->tileB8[prec], &A->ntileB8[prec], st));
    PP_TRY(build_round_plan(A, prec, 16, &A->tileB16[prec], &A->ntileB16[prec], st));
    const Workspace &w = A->ws[prec];
    HIP_TRY(hipMemsetAsync(w.P0, 0, (size_t)w.ldv * elem_size(prec), st));
    HIP_TRY(hipMemsetAsync(w.P1, 0, (size_t)w.ldv * elem_size(prec), st));
    StepPtrs p;
    std::memset(&p, 0, sizeof(p));
    p.in = w.P0;
    p.out = w.P1;
    p.spmv = 1;
    p.a0 = 1.0;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    double best = 1e30;
    int bv = CV_TILE8, br = 1;
    // every (variant, remap) is timed over `reps` launches in two rounds and
    // keeps its faster round, so one noisy trial does not decide the pick
    const int reps = 10;
    for (int round = 0; round < 2; ++round)
    for (int v = 0; v < CV_COUNT; ++v) {
        if (v == CV_PERSIST || ((v == CV_SELL || v == CV_SELLT || v == CV_SELL2 || v == CV_SELL4) && A->nslices == 0) ||
            ((v == CV_SELLD || v == CV_SELLD4) && !A->sdel) || ((v == CV_DIA || v == CV_DIA4) && A->h_doff.empty()) ||
            (v == CV_DIAC && !A->dcode) || (v == CV_DIAP && !A->pcode) || (v == CV_DIAPV && !A->pbyte) ||
            (v == CV_BAND2 && A->bandK[0] == 0) || (v == CV_BAND4 && A->bandK[1] == 0) ||
            ((v == CV_CSORT4 || v == CV_CSORT2) && A->cs_nb == 0) ||
            (v == CV_TILEB8 && A->ntileB8[prec] == 0) ||
            (v == CV_TILEB16 && A->ntileB16[prec] == 0) || (v == CV_BOX && !box_step_ok(A->dev())))
            continue;
        for (int r = 0; r < 2; ++r) {
            A->variant[prec] = v;
            A->remap[prec] = r;
            const DevCSR d = A->dev();
            for (int i = 0; i < 2; ++i) HIP_TRY(launch_chain_step(d, prec, p, st));
            HIP_TRY(hipEventRecord(e0, st));
            for (int i = 0; i < reps; ++i) HIP_TRY(launch_chain_step(d, prec, p, st));
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * ms / reps;
            if (us < best) {
                best = us;
                bv = v;
                br = r;
            }
        }
    }
    A->variant[prec] = bv;
    A->remap[prec] = br;
    A->persist[prec] = 0;
    double best_all = best;
    // two steps per launch on a box stencil (the pairs that chains with an
    // accumulator use: p chains' steps): one such launch, with the cube-tile
    // kernel or whole-line tiles where they apply, against two single steps
    // that also read and write the accumulator; kept when it is faster
    A->fuse[prec] = 0;
    A->pair_us[prec] = 0.0;
    A->pair_tile[prec] = 0;
    if (A->box_nd && A->pbyte && prec != PP_BF16S) {
        const DevCSR d = A->dev();
        auto timed = [&](auto &&launch, double &best_us) -> pp_status {
            for (int round = 0; round < 2; ++round) {
                for (int i = 0; i < 2; ++i) HIP_TRY(launch());
                HIP_TRY(hipEventRecord(e0, st));
                for (int i = 0; i < reps; ++i) HIP_TRY(launch());
                HIP_TRY(hipEventRecord(e1, st));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                best_us = std::min(best_us, 1e3 * ms / reps);
            }
            return PP_OK;
        };
        StepPtrs sa = p;
        sa.acc = w.T;
        sa.b0 = sa.b1 = 1.0;
        double single_acc = 1e30;
        PP_TRY(timed([&] { return launch_chain_step(d, prec, sa, st); }, single_acc));
        PairPtrs pp;
        std::memset(&pp, 0, sizeof(pp));
        pp.in = w.P0;
        pp.out = w.P1;
        pp.acc = w.T;
        pp.acc1 = pp.acc2 = 1;
        pp.a01 = pp.a02 = 1.0;
        pp.b01 = pp.b11 = pp.b02 = pp.b12 = 1.0;
        double bp = 1e30;
        PP_TRY(timed([&] { return launch_chain_pair(d, prec, pp, br, st); }, bp));
        if (box_tile_ok(d, prec)) {
            PairPtrs tp = pp;
            tp.shape = 1;
            for (int r = 0; r < 2; ++r) {
                double bt = 1e30;
                PP_TRY(timed([&] { return launch_chain_pair(d, prec, tp, r, st); }, bt));
                if (bt < bp) {
                    bp = bt;
                    A->pair_tile[prec] = 1;
                    A->pair_remap[prec] = r;
                }
            }
        }
        A->pair_us[prec] = bp;
        A->fuse[prec] = bp < 2.0 * single_acc ? 1 : 0;
    }
    // 2 to kMarchMax steps per launch of the marching kernel: each launch
    // length is timed over a few plane-chunk sizes; the length with the
    // lowest time per step is kept when it beats a single step
    A->march[prec] = 0;
    A->march_all[prec] = 0;
    A->march_tile[prec] = 0;
    for (int g = 0; g <= kMarchMax; ++g) {
        A->march_us[prec][g] = 0.0;
        A->march_cz[prec][g] = 0;
    }
    if (A->box_nd && A->pbyte && prec != PP_BF16S) {
        const DevCSR d = A->dev();
        MarchPtrs mp;
        std::memset(&mp, 0, sizeof(mp));
        mp.in = w.P0;
        mp.out = w.P1;
        for (int k = 0; k < kMarchMax; ++k) mp.a0[k] = 1.0;
        const int cz0 = march_default_cz(d, 1024);
        const int czs[3] = {cz0, 2 * cz0, std::max(4, cz0 / 2)};
        const int ndepth = A->box_pint >= 0 ? 3 : 1;  // deeper prefetch: constant-coefficient kernels only
        double per_step = best;
        for (int g = 2; g <= kMarchMax; ++g) {
            mp.nsteps = g;
            double bg = 1e30;
            int bcz = cz0, bdepth = 1;
            for (int c = 0; c < 3; ++c) {
                if (c > 0 && (czs[c] == czs[0] || (c == 2 && czs[2] == czs[1]))) continue;
                for (int depth = 1; depth <= ndepth; ++depth) {
                    mp.depth = depth;
                    for (int round = 0; round < 2; ++round) {
                        for (int i = 0; i < 2; ++i) HIP_TRY(launch_chain_march(d, prec, mp, czs[c], br, st));
                        HIP_TRY(hipEventRecord(e0, st));
                        for (int i = 0; i < reps; ++i) HIP_TRY(launch_chain_march(d, prec, mp, czs[c], br, st));
                        HIP_TRY(hipEventRecord(e1, st));
                        HIP_TRY(hipEventSynchronize(e1));
                        float ms = 0.f;
                        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                        const double us = 1e3 * ms / reps;
                        if (us < bg) {
                            bg = us;
                            bcz = czs[c];
                            bdepth = depth;
                        }
                    }
                }
            }
            // two steps: whole-line tiles instead of marching planes, where
            // they apply and are faster
            if (g == 2 && box_tile_ok(d, prec)) {
                MarchPtrs tp = mp;
                tp.shape = 1;
                tp.depth = 0;
                double bt = 1e30;
                for (int round = 0; round < 2; ++round)
                    for (int r = 0; r < 2; ++r) {
                        for (int i = 0; i < 2; ++i) HIP_TRY(launch_chain_march(d, prec, tp, 0, r, st));
                        HIP_TRY(hipEventRecord(e0, st));
                        for (int i = 0; i < reps; ++i) HIP_TRY(launch_chain_march(d, prec, tp, 0, r, st));
                        HIP_TRY(hipEventRecord(e1, st));
                        HIP_TRY(hipEventSynchronize(e1));
                        float ms = 0.f;
                        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                        const double us = 1e3 * ms / reps;
                        if (us < bt) {
                            bt = us;
                            A->tile_remap[prec] = r;
                        }
                    }
                if (bt < bg) {
                    bg = bt;
                    A->march_tile[prec] = 1;
                }
            }
            A->march_us[prec][g] = bg;
            A->march_cz[prec][g] = bcz;
            A->march_depth[prec][g] = bdepth;
            if (bg / g < per_step) {
                per_step = bg / g;
                A->march[prec] = g;
            }
        }
    }
    // The persistent kernel is only timed on request: its grid barrier must
    // write back and invalidate the per-XCD L2 caches, which costs far more
    // than a kernel boundary on this GPU.
    if (A->pgrid > 0 && A->tune_persist) {
        for (int r = 0; r < 2; ++r) {
            PP_TRY(launch_persist(A, prec, A->tune_steps, 8, w.P0, w.P1, r, st));
            HIP_TRY(hipEventRecord(e0, st));
            for (int i = 0; i < 2; ++i) PP_TRY(launch_persist(A, prec, A->tune_steps, 8, w.P0, w.P1, r, st));
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            HIP_TRY(copy_barrier_flag(A, st));
            HIP_TRY(hipStreamSynchronize(st));
            PP_TRY(check_barrier_flag(A));
            const double us = 1e3 * ms / (2 * 8);
            if (us < best_all) {
                best_all = us;
                A->persist[prec] = 1;
                A->premap[prec] = r;
            }
        }
    }
    A->tuned[prec] = 1;
    A->tuned_us[prec] = best_all;
    return PP_OK;
}

pp_status ensure_tuned(pp_matrix A, int prec, hipStream_t st) {
    if (A->tuned[prec]) return PP_OK;
    return tune_chain(A, prec, st);
}

const std::vector<Step> &prog_of(pp_poly p, int kind) {
    return kind == PP_APPLY_P ? p->prog_p : (kind == PP_APPLY_PHI ? p->prog_phi : p->prog_pi);
}

// Evaluate a chain program: one cooperative launch (persistent kernel) or
// one launch per step, as tuned for this matrix and precision.
pp_status run_composite(pp_matrix A, pp_poly poly, int kind, int prec, const void *in, void *out, hipStream_t st);

// Steps i and i+1 of a chain program can run as one fused pair: both one
// sparse product, the first without an aux vector, the second reading the
// first's result and at most the first's input as aux (a conjugate pair's
// second step); nothing later reads the first's result before it is
// written again; at most one accumulator, updated by the second step only
// when the first's initialisation came before it.
bool pair_fusable(const std::vector<Step> &prog, size_t i) {
    const Step &s = prog[i], &t = prog[i + 1];
    if (s.spmv != 1 || t.spmv != 1 || s.aux != B_NONE || (t.aux != B_NONE && t.aux != s.in) || s.fin) return false;
    if (s.out < B_P0 || t.in != s.out || t.out == s.out || t.out == B_IN) return false;
    if (s.acc != B_NONE && t.acc != B_NONE && (s.acc != t.acc || t.acc_init)) return false;
    const int acc = s.acc != B_NONE ? s.acc : t.acc;
    if (acc != B_NONE && (acc == s.in || acc == s.out || acc == t.out)) return false;
    for (size_t j = i + 2; j < prog.size(); ++j) {
        const Step &u = prog[j];
        if (u.in == s.out || u.aux == s.out || (u.acc == s.out && !u.acc_init)) return false;
        if (u.out == s.out || u.acc == s.out) break;
    }
    return true;
}

// Steps i .. i+g-1 of a chain program can run as one launch of the
// marching kernel: each one sparse product without an accumulator; the
// first without aux; each later one reading the previous step's result and,
// as aux, at most the previous step's input (a conjugate pair's second
// step); every result but the last a temporary without a final vector; and
// no intermediate result read after the group before it is written again.
bool march_group_ok(const std::vector<Step> &prog, size_t i, int g) {
    const size_t last = i + g - 1;
    for (size_t k = i; k < last; ++k) {
        const int b = prog[k].out;
        bool rewritten = false;
        for (size_t m = k + 1; m <= last; ++m)
            if (prog[m].out == b) {
                rewritten = true;
                break;
            }
        if (rewritten) continue;
        for (size_t j = last + 1; j < prog.size(); ++j) {
            const Step &u = prog[j];
            if (u.in == b || u.aux == b || (u.acc == b && !u.acc_init)) return false;
            if (u.out == b || u.acc == b) break;
        }
    }
    return true;
}

int march_group_len(const std::vector<Step> &prog, size_t i, int smax) {
    const Step &s0 = prog[i];
    if (s0.spmv != 1 || s0.acc != B_NONE || s0.aux != B_NONE || s0.out == B_NONE || s0.out == s0.in) return 1;
    int g = 1;
    while (g < smax && i + g < prog.size()) {
        const Step &p = prog[i + g - 1], &t = prog[i + g];
        if (p.fin || p.out < B_P0) break;
        if (t.spmv != 1 || t.acc != B_NONE || t.in != p.out || t.out == B_NONE || t.out == t.in) break;
        if (t.aux != B_NONE && t.aux != p.in) break;
        ++g;
    }
    for (; g >= 2; --g)
        if (march_group_ok(prog, i, g)) break;
    return g;
}

// One launch of a chain program as run_program issues it.
struct Planned {
    int kind;   // 0: one step, 1: the two-step pair kernel, 2: the marching kernel
    int i, g;   // steps i .. i+g-1
    int write;  // the buffer the launch's last result goes to
    int swap;   // after the launch the names `write` and the last step's out swap (-1: no swap)
};

// The launches of a chain program with this matrix's fusion settings for the
// precision. A fused launch reads its input around its tile while other
// workgroups write: when its last step's output buffer is the group's input
// (ping-pong temporaries), the result goes to a temporary whose value is
// dead after the group and the two names swap for the rest of the program.
void plan_program(pp_matrix A, const std::vector<Step> &prog, int prec, std::vector<Planned> &out) {
    out.clear();
    const bool coded = A->box_nd && A->pbyte && prec != PP_BF16S && !A->persist[prec];
    const bool pair = coded && A->fuse[prec];
    const int smax = coded ? A->march[prec] : 0;
    for (size_t i = 0; i < prog.size();) {
        const Step &s = prog[i];
        if (smax >= 2) {
            int g = march_group_len(prog, i, smax);
            // a shorter group runs only if that launch length beats single steps
            while (g >= 2 && g < smax && !A->march_all[prec] &&
                   !(A->march_us[prec][g] > 0.0 && A->march_us[prec][g] < g * A->tuned_us[prec]))
                --g;
            if (g >= 2) {
                const Step &t = prog[i + g - 1];
                Planned L{2, (int)i, g, t.out, -1};
                if (t.out == s.in) {
                    L.write = s.out;  // step i's result: a temporary, dead after the group
                    L.swap = s.out;
                }
                out.push_back(L);
                i += g;
                continue;
            }
        }
        if (pair && i + 1 < prog.size() && pair_fusable(prog, i)) {
            const Step &t = prog[i + 1];
            const bool swap = t.out != B_NONE && t.out == s.in && s.out >= B_P0 && t.out >= B_P0;
            const int write = swap ? s.out : t.out;
            const int acc = s.acc != B_NONE ? s.acc : t.acc;
            if (write != s.in && (acc == B_NONE || acc != s.in)) {
                out.push_back(Planned{1, (int)i, 2, write, swap ? s.out : -1});
                i += 2;
                continue;
            }
        }
        out.push_back(Planned{0, (int)i, 1, s.out, -1});
        ++i;
    }
}

// temps: the three temporary vectors (B_P0, B_P1, B_T) of the program; null
// for the handle's workspace of this precision.
pp_status run_program(pp_matrix A, pp_poly poly, int kind, int prec, const void *in, void *out, hipStream_t st,
                      void *const *temps = nullptr) {
    if (poly->inner) return run_composite(A, poly, kind, prec, in, out, st);
    PP_TRY(ensure_tuned(A, prec, st));
    const std::vector<Step> &prog = prog_of(poly, kind);
    if (A->persist[prec] && prog.size() >= 2) {
        const auto key = std::make_pair((unsigned long long)poly->id, kind);
        auto it = A->progs.find(key);
        PStep *table = nullptr;
        if (it == A->progs.end()) {
            std::vector<PStep> h;
            for (const Step &s : prog) h.push_back(to_pstep(s));
            PP_TRY(upload_steps(h, &table, st));
            A->progs[key] = table;
        } else {
            table = it->second;
        }
        return launch_persist(A, prec, table, (int)prog.size(), in, out, A->premap[prec], st);
    }
    const Workspace &w = A->ws[prec];
    const DevCSR d = A->dev();
    // The temporaries' buffers; a fused launch may swap two of them.
    void *tmp[5] = {nullptr, nullptr, temps ? temps[0] : w.P0, temps ? temps[1] : w.P1, temps ? temps[2] : w.T};
    auto ptr = [&](int b) -> void * {
        if (b == B_IN) return (void *)in;
        if (b == B_OUT) return out;
        return b >= B_P0 && b <= B_T ? tmp[b] : nullptr;
    };
    std::vector<Planned> plan;
    plan_program(A, prog, prec, plan);
    for (const Planned &L : plan) {
        const Step &s = prog[L.i];
        if (L.kind == 2) {
            const Step &t = prog[L.i + L.g - 1];
            MarchPtrs mp;
            std::memset(&mp, 0, sizeof(mp));
            mp.in = ptr(s.in);
            mp.out = ptr(L.write);
            mp.vfin = t.fin ? in : nullptr;
            mp.nsteps = L.g;
            for (int k = 0; k < L.g; ++k) {
                const Step &u = prog[L.i + k];
                mp.a0[k] = u.a0;
                mp.a1[k] = u.a1;
                mp.a2[k] = u.a2;
                if (u.aux != B_NONE) mp.aux |= 1 << k;
            }
            mp.depth = A->march_depth[prec][L.g];
            mp.shape = L.g == 2 && A->march_tile[prec] ? 1 : 0;
            HIP_TRY(launch_chain_march(d, prec, mp, A->march_cz[prec][L.g],
                                       mp.shape ? A->tile_remap[prec] : A->remap[prec], st));
            if (L.swap >= 0) std::swap(tmp[L.swap], tmp[t.out]);
            continue;
        }
        if (L.kind == 1) {
            // Two real-root steps in one launch. The first step's result is
            // not stored.
            const Step &t = prog[L.i + 1];
            PairPtrs pp;
            pp.in = ptr(s.in);
            pp.out = ptr(L.write);
            pp.acc = ptr(s.acc != B_NONE ? s.acc : t.acc);
            pp.vfin = t.fin ? in : nullptr;
            pp.acc1 = s.acc != B_NONE;
            pp.acc2 = t.acc != B_NONE;
            pp.init = s.acc != B_NONE ? s.acc_init : t.acc_init;
            pp.aux2 = t.aux != B_NONE;
            pp.a22 = t.a2;
            pp.a01 = s.a0;
            pp.a11 = s.a1;
            pp.b01 = s.b0;
            pp.b11 = s.b1;
            pp.a02 = t.a0;
            pp.a12 = t.a1;
            pp.b02 = t.b0;
            pp.b12 = t.b1;
            pp.shape = A->pair_tile[prec];
            HIP_TRY(launch_chain_pair(d, prec, pp, pp.shape ? A->pair_remap[prec] : A->remap[prec], st));
            if (L.swap >= 0) std::swap(tmp[L.swap], tmp[t.out]);
            continue;
        }
        StepPtrs p;
        p.in = ptr(s.in);
        p.aux = ptr(s.aux);
        p.vfin = s.fin ? in : nullptr;
        p.out = ptr(s.out);
        p.acc = ptr(s.acc);
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

// A composite polynomial phi2(phi1(A)) (section 6). The outer program is
// phi2's with every sparse product replaced by phi1(A): the inner chain
// writes phi1(A) in into Q, then one elementwise launch applies the outer
// step's update with Q as its product term. kind P: p1(A) p2(phi1(A)) v,
// the outer p2 program into E, then the inner p1 program from E.
pp_status run_composite(pp_matrix A, pp_poly poly, int kind, int prec, const void *in, void *out, hipStream_t st) {
    PP_TRY(ensure_tuned(A, prec, st));
    PP_TRY(A->ensure_extra(prec));
    const Workspace &w = A->ws[prec];
    const size_t vec = (size_t)w.ldv * elem_size(prec);
    char *X = (char *)w.X;
    void *Q = X, *O0 = X + vec, *O1 = X + 2 * vec, *OT = X + 3 * vec, *E = X + 4 * vec;
    pp_poly inner = const_cast<pp_poly>(poly->inner.get());
    void *dst = kind == PP_APPLY_P ? E : out;
    auto bp = [&](int b) -> void * {
        switch (b) {
            case B_IN:
                return (void *)in;
            case B_OUT:
                return dst;
            case B_P0:
                return O0;
            case B_P1:
                return O1;
            case B_T:
                return OT;
            default:
                return nullptr;
        }
    };
    for (const Step &s : prog_of(poly, kind)) {
        StepPtrs p;
        p.in = bp(s.in);
        p.aux = bp(s.aux);
        p.vfin = s.fin ? in : nullptr;
        p.out = bp(s.out);
        p.acc = bp(s.acc);
        p.acc_init = s.acc_init;
        p.spmv = 0;
        p.a0 = s.a0;
        p.a1 = s.a1;
        p.a2 = s.a2;
        p.b0 = s.b0;
        p.b1 = s.b1;
        p.prod = nullptr;
        if (s.spmv) {
            PP_TRY(run_program(A, inner, PP_APPLY_PHI, prec, p.in, Q, st));
            p.prod = Q;
        }
        HIP_TRY(launch_chain_step(A->dev(), prec, p, st));
    }
    if (kind == PP_APPLY_P) PP_TRY(run_program(A, inner, PP_APPLY_P, prec, E, out, st));
    return PP_OK;
}

// Device-memory bytes of one sparse product's matrix data in the format the
// chain variant of this precision reads: stored values and indices (or codes,
// or row patterns and their table), row pointers or slice offsets; for the
// column-banded copies also the partial row sums passed from one band to the
// next (written by all bands but the last, read by all but the first).
int64_t format_bytes(pp_matrix A, int prec) {
    const int64_t n = A->n, nnz = A->nnz;
    const int64_t sv = prec == PP_F64 ? 8 : 4;  // matrix values: binary64, else binary32
    const int64_t nd = (int64_t)A->h_doff.size();
    switch (A->variant[prec]) {
        case CV_SELL:
        case CV_SELLT:
        case CV_SELL2:
        case CV_SELL4:
            return (int64_t)A->npad * (sv + 4) + 4 * ((int64_t)A->nslices + 1);
        case CV_SELLD:
        case CV_SELLD4:
            return (int64_t)A->npad * (sv + 2) + 4 * ((int64_t)A->nslices + 1);
        case CV_DIA:
        case CV_DIA4:
            return (n + 255) / 256 * 256 * nd * sv;
        case CV_DIAC:
            return n * ((nd + 7) / 8) * 8 + (int64_t)A->ntab * sv;
        case CV_DIAP:
        case CV_DIAPV:
            return n + (int64_t)A->npat * nd * sv;
        case CV_BOX:  // the interior row's coefficients only
            return nd * sv;
        case CV_BAND2:
        case CV_BAND4: {
            const int c = A->variant[prec] == CV_BAND2 ? 0 : 1;
            const int64_t K = A->bandK[c];
            return (int64_t)A->bnnz[c] * (sv + 4) + K * 4 * (n + 1) + (K - 1) * 2 * n * sv;
        }
        case CV_CSORT4:
        case CV_CSORT2: {
            // tile entries (word + value), tile row pointers and offsets, the
            // held-apart diagonal, each partial sum written and read
            const int64_t nsb = A->variant[prec] == CV_CSORT4 ? 4 : 2;
            const int64_t nt = (n + kCsRows - 1) / kCsRows * A->cs_nb;
            return (int64_t)A->cs_nnz * (sv + 4) + nt * (kCsRows + 1) * 2 + (nt + 1) * 4 +
                   (A->cs_dperm ? n * sv : 0) + 2 * nsb * n * sv;
        }
        default:  // CSR: row tiles, lanes per row, persistent
            return nnz * (sv + 4) + 4 * (n + 1);
    }
}

// Launches of one sparse product with the chain variant of this precision.
int64_t product_launches(pp_matrix A, int prec) {
    const int v = A->variant[prec];
    if (v == CV_BAND2 || v == CV_BAND4) return A->bandK[v == CV_BAND2 ? 0 : 1];
    if (v == CV_CSORT4 || v == CV_CSORT2) return 2;
    return 1;
}

// The bytes and launches of one application of a chain program, walked as
// run_program runs it (the same two-step fusion), without launching: per
// launch the matrix data of its sparse products, one read of the input, the
// aux and final vectors, the accumulator (read unless initialised, written)
// and one write of the output; a fused pair reads its input and matrix data
// once and never stores the first step's result.
void program_bytes(pp_matrix A, pp_poly poly, int kind, int prec, int64_t &bytes, int64_t &launches) {
    const int64_t vec = (int64_t)A->n * (int64_t)elem_size(prec);
    const int64_t fmt = format_bytes(A, prec);
    const std::vector<Step> &prog = prog_of(poly, kind);
    if (poly->inner) {
        pp_poly in = const_cast<pp_poly>(poly->inner.get());
        for (const Step &s : prog) {
            if (s.spmv) program_bytes(A, in, PP_APPLY_PHI, prec, bytes, launches);
            bytes += vec * (1 + (s.spmv ? 1 : 0) + (s.aux != B_NONE) + (s.fin != 0) + (s.out != B_NONE));
            if (s.acc != B_NONE) bytes += vec * (s.acc_init ? 1 : 2);
            launches += 1;
        }
        if (kind == PP_APPLY_P) program_bytes(A, in, PP_APPLY_P, prec, bytes, launches);
        return;
    }
    // fused launches read the pattern-coded copy, whatever the single-step
    // variant; on a constant-coefficient stencil only the interior row's
    // coefficients
    const int64_t csz = prec == PP_F64 ? 8 : 4;
    const int64_t coded = (int64_t)A->n + (int64_t)A->npat * (int64_t)A->h_doff.size() * csz;
    const int64_t pat = A->box_pint >= 0 ? (int64_t)A->h_doff.size() * csz : coded;
    // the cube-tile pair kernel reads the pattern bytes on any box stencil
    const int64_t pat_pair = A->pair_tile[prec] ? pat : coded;
    std::vector<Planned> plan;
    plan_program(A, prog, prec, plan);
    for (const Planned &L : plan) {
        const Step &s = prog[L.i], &t = prog[L.i + L.g - 1];
        if (L.kind == 2) {
            // the input and the pattern bytes once, the final vector, the output
            bytes += pat + vec * (1 + (t.fin != 0) + 1);
            launches += 1;
            continue;
        }
        if (L.kind == 1) {
            const int acc = s.acc != B_NONE ? s.acc : t.acc;
            const int init = s.acc != B_NONE ? s.acc_init : t.acc_init;
            bytes += pat_pair + vec * (1 + (t.out != B_NONE) + (t.fin != 0));
            if (acc != B_NONE) bytes += vec * (init ? 1 : 2);
            launches += 1;
            continue;
        }
        if (s.spmv) {
            bytes += fmt;
            launches += product_launches(A, prec);
        } else {
            launches += 1;
        }
        bytes += vec * (1 + (s.aux != B_NONE) + (s.fin != 0) + (s.out != B_NONE));
        if (s.acc != B_NONE) bytes += vec * (s.acc_init ? 1 : 2);
    }
    if (A->persist[prec] && prog.size() >= 2) launches -= (int64_t)prog.size() - 1;  // one cooperative launch
}

// Scratch of pp_apply_noalloc: the chain's three temporary vectors, in a
// file-scope device array that each GPU the library runs on holds until the
// process ends. Host code must not pass the array's name to a kernel (on the
// host it is a stand-in, not a device address): its device address is taken
// once per device with hipGetSymbolAddress and used instead.
constexpr size_t kNoallocScratchBytes = (size_t)3 * 2097152 * 8;  // 48 MiB: FP64 n <= 2^21
constexpr int kNoallocMaxDevices = 64;
__device__ __align__(256) unsigned char noalloc_scratch_mem[kNoallocScratchBytes];
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoallocMaxDevices] = {};

// The scratch array's device address on the current device (looked up on the
// first call on that device, with the device current).
pp_status noalloc_scratch(char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) {
        set_error("pp_apply_noalloc: device index out of range");
        return PP_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch_mem));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("pp_apply_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
            return PP_EDEVICE;
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = (char *)g_noalloc_ptr[dev];
    return PP_OK;
}

// Sparse products of one application of a polynomial (kind PHI/PI or P).
int64_t chain_mvps(pp_poly p, int kind) {
    if (!p->inner) return kind == PP_APPLY_P ? p->plan.d_eff - 1 : p->plan.d_eff;
    const int64_t inner_phi = chain_mvps(const_cast<pp_poly>(p->inner.get()), PP_APPLY_PHI);
    const int64_t outer = kind == PP_APPLY_P ? p->plan.d_eff - 1 : p->plan.d_eff;
    return outer * inner_phi +
           (kind == PP_APPLY_P ? chain_mvps(const_cast<pp_poly>(p->inner.get()), PP_APPLY_P) : 0);
}

// Launches of one application (for the vector-operation counter).
int64_t chain_launches(pp_poly p, int kind) {
    const std::vector<Step> &prog = prog_of(p, kind);
    if (!p->inner) return (int64_t)prog.size();
    const pp_poly in = const_cast<pp_poly>(p->inner.get());
    int64_t n = 0;
    for (const Step &s : prog) n += 1 + (s.spmv ? chain_launches(in, PP_APPLY_PHI) : 0);
    return n + (kind == PP_APPLY_P ? chain_launches(in, PP_APPLY_P) : 0);
}

// One step of the SpMV alone: out = a0 * A in + a2 * aux
pp_status spmv_axpby(pp_matrix A, int prec, const void *in, double a0, const void *aux, double a2, void *out,
                     hipStream_t st) {
    PP_TRY(ensure_tuned(A, prec, st));
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
pp_status cgs2_step(pp_matrix A, int prec, const Workspace &ws, int j, hipStream_t st, double *Hcol = nullptr,
                    bool to_host = true) {
    if (!Hcol) Hcol = A->H();
    const int n = A->n;
    const int ncols = j + 1;
    void *w = vcol(ws, prec, j + 1);
    // pass 1: h1 = V^T w
    HIP_TRY(launch_dots(prec, n, ws.V, ws.ldv, ncols, w, A->partial, A->ldp, st));
    HIP_TRY(launch_reduce(A->nblk_dot, A->partial, A->ldp, ncols, A->h1(), Hcol, 1, st));
    // w -= V h1 ; h2 = V^T w and ||w||^2 (one read of V when the row fits in
    // registers); then w = (w - V h2) / ||w - V h2|| in one more pass, the
    // norm following from ||w||^2 - ||h2||^2
    if (ncols <= update_dots_max_cols(prec)) {
        HIP_TRY(launch_update_dots(prec, n, ws.V, ws.ldv, ncols, A->h1(), w, A->partial, A->ldp, st));
        HIP_TRY(launch_reduce(A->nblk_ud, A->partial, A->ldp, ncols + 1, A->h2(), nullptr, 0, st));
        HIP_TRY(launch_finish_col(ncols, A->h2(), Hcol, A->inv(), st));
        HIP_TRY(launch_update_scale(prec, n, ws.V, ws.ldv, ncols, A->h2(), w, A->inv(), st));
    } else {
        HIP_TRY(launch_update(prec, n, ws.V, ws.ldv, ncols, A->h1(), w, nullptr, st));
        HIP_TRY(launch_dots(prec, n, ws.V, ws.ldv, ncols, w, A->partial, A->ldp, st));
        HIP_TRY(launch_reduce(A->nblk_dot, A->partial, A->ldp, ncols, A->h2(), Hcol, 2, st));
        // w -= V h2 ; ||w|| ; w /= ||w||
        HIP_TRY(launch_update(prec, n, ws.V, ws.ldv, ncols, A->h2(), w, A->npart, st));
        HIP_TRY(launch_reduce_norm(A->nblk_upd, A->npart, Hcol + ncols, A->inv(), st));
        HIP_TRY(launch_scale_cast(prec, prec, n, w, A->inv(), 0.0, w, st));
    }
    if (!to_host) return PP_OK;
    HIP_TRY(hipMemcpyAsync(A->hpin, Hcol, sizeof(double) * (ncols + 1), hipMemcpyDeviceToHost, st));
    HIP_TRY(copy_barrier_flag(A, st));
    HIP_TRY(hipStreamSynchronize(st));
    return check_barrier_flag(A);
}

// ||x|| of a device vector (synchronises); x is not modified.
pp_status dev_norm(pp_matrix A, int prec, const void *x, double *out, hipStream_t st) {
    HIP_TRY(launch_dots(prec, A->n, x, 0, 1, x, A->partial, A->ldp, st));
    HIP_TRY(launch_reduce(A->nblk_dot, A->partial, A->ldp, 1, A->h1(), nullptr, 0, st));
    HIP_TRY(hipMemcpyAsync(A->hpin, A->h1(), sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(copy_barrier_flag(A, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(A->hpin[0]);
    return check_barrier_flag(A);
}

bool valid_prec(int p) { return p >= 0 && p <= 2; }

// Column-banded CSR copy c with K bands: band k holds the entries whose
// column lies in [k n / K, (k+1) n / K), in CSR order, with its own row
// pointers (offsets into the shared entry arrays) and 256-row tiles of at
// most 2044 entries.
pp_status build_bands(pp_matrix A, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, const double *val,
                      int c, int K, hipStream_t st) {
    const int64_t n = A->n, nnz = A->nnz;
    std::vector<int32_t> brp((size_t)K * (n + 1)), bc(nnz), bp(nnz);
    std::vector<int64_t> cnt(K, 0);
    for (int64_t e = 0; e < nnz; ++e) cnt[(int)((int64_t)ci[e] * K / n)]++;
    std::vector<int64_t> start(K + 1, 0);
    for (int k = 0; k < K; ++k) start[k + 1] = start[k] + cnt[k];
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t r = 0; r < n; ++r) {
        for (int k = 0; k < K; ++k) brp[(size_t)k * (n + 1) + r] = (int32_t)pos[k];
        for (int e = rp[r]; e < rp[r + 1]; ++e) {
            const int k = (int)((int64_t)ci[e] * K / n);
            bc[pos[k]] = ci[e];
            bp[pos[k]] = e;
            ++pos[k];
        }
    }
    for (int k = 0; k < K; ++k) brp[(size_t)k * (n + 1) + n] = (int32_t)pos[k];
    std::vector<int4> tiles, t;
    A->btoff[c][0] = 0;
    for (int k = 0; k < K; ++k) {
        build_tiles(brp.data() + (size_t)k * (n + 1), (int)n, 256, 256 * 8 - 4, t);
        tiles.insert(tiles.end(), t.begin(), t.end());
        A->btoff[c][k + 1] = (int)tiles.size();
    }
    PP_TRY(dev_alloc(&A->brow[c], brp.size()));
    PP_TRY(dev_alloc(&A->bcol[c], (size_t)nnz));
    PP_TRY(dev_alloc(&A->bperm[c], (size_t)nnz));
    PP_TRY(dev_alloc(&A->bval64[c], (size_t)nnz));
    PP_TRY(dev_alloc(&A->bval32[c], (size_t)nnz));
    PP_TRY(dev_alloc(&A->btile[c], tiles.size()));
    if (!A->bpart) PP_TRY(dev_alloc(&A->bpart, (size_t)n));
    if (hipMemcpyAsync(A->brow[c], brp.data(), sizeof(int32_t) * brp.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(A->bcol[c], bc.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(A->bperm[c], bp.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(A->btile[c], tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        launch_sell_values(nnz, A->bperm[c], val, A->bval64[c], A->bval32[c], st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("pp_matrix_create: column-banded upload failed");
        return PP_EDEVICE;
    }
    A->bnnz[c] = nnz;
    A->bandK[c] = K;
    return PP_OK;
}

// Column-sorted tiles (the layout is described with DevCSR). The band count
// is the smallest of 16, 32, 64, 128 for which every band is non-empty and
// every tile fits: at most 65535 entries, its FP64 products in 80 KB of LDS
// (two workgroups per CU), column offset and slot in one 32-bit word. When
// none fits the matrix has no such copy. The diagonal is held apart when
// every row stores exactly one diagonal entry. Blocks are laid out on
// several host threads.
pp_status build_csort(pp_matrix A, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, const double *val,
                      hipStream_t st) {
    const int64_t n = A->n;
    const int nblk = (int)((n + kCsRows - 1) / kCsRows);
    std::vector<int32_t> dpos((size_t)n, -1);
    bool split = true;
    for (int64_t r = 0; r < n && split; ++r)
        for (int e = rp[r]; e < rp[r + 1]; ++e)
            if (ci[e] == r) {
                if (dpos[r] >= 0) split = false;
                dpos[r] = e;
            }
    for (int64_t r = 0; r < n && split; ++r)
        if (dpos[r] < 0) split = false;
    int nb = 0, sb = 0;
    int64_t W = 0, maxe = 0;
    std::vector<int64_t> cnt;
    for (int cand : {16, 32, 64, 128}) {
        const int64_t w = (n + cand - 1) / cand;
        if ((cand - 1) * w >= n) continue;  // the last band would be empty
        cnt.assign((size_t)nblk * cand, 0);
        for (int64_t r = 0; r < n; ++r)
            for (int e = rp[r]; e < rp[r + 1]; ++e)
                if (!(split && e == dpos[r])) cnt[(size_t)(r / kCsRows) * cand + ci[e] / w]++;
        int64_t mx = 1;
        for (int64_t c : cnt) mx = std::max(mx, c);
        int bits = 1, cbits = 0;
        while ((int64_t(1) << bits) < mx) ++bits;
        while ((int64_t(1) << cbits) < w) ++cbits;
        if (mx <= 65535 && mx * 8 <= kCsLdsBytes && bits + cbits <= 32) {
            nb = cand;
            sb = bits;
            W = w;
            maxe = mx;
            break;
        }
    }
    if (nb == 0) return PP_OK;
    const size_t nt = (size_t)nblk * nb;
    std::vector<int32_t> toff(nt + 1, 0);
    for (size_t t = 0; t < nt; ++t) toff[t + 1] = toff[t] + (int32_t)cnt[t];
    const int64_t ne = toff[nt];
    std::vector<uint32_t> code((size_t)ne);
    std::vector<int32_t> perm((size_t)ne);
    std::vector<uint16_t> tptr(nt * (kCsRows + 1));
    auto lay_block = [&](int b) {
        const int64_t r0 = (int64_t)b * kCsRows, r1 = std::min<int64_t>(n, r0 + kCsRows);
        std::vector<int32_t> run(nb, 0);
        std::vector<std::vector<std::pair<uint64_t, int32_t>>> ent(nb);  // (column << 20 | slot, CSR index)
        for (int c = 0; c < nb; ++c) ent[c].reserve((size_t)cnt[(size_t)b * nb + c]);
        for (int64_t r = r0; r < r1; ++r) {
            for (int c = 0; c < nb; ++c) tptr[((size_t)b * nb + c) * (kCsRows + 1) + (r - r0)] = (uint16_t)run[c];
            for (int e = rp[r]; e < rp[r + 1]; ++e) {
                if (split && e == dpos[r]) continue;
                const int c = (int)(ci[e] / W);
                ent[c].push_back({((uint64_t)ci[e] << 20) | (uint64_t)run[c], e});
                ++run[c];
            }
        }
        for (int c = 0; c < nb; ++c) {
            const size_t t = (size_t)b * nb + c;
            for (int64_t rl = r1 - r0; rl <= kCsRows; ++rl) tptr[t * (kCsRows + 1) + rl] = (uint16_t)run[c];
            std::sort(ent[c].begin(), ent[c].end());
            for (size_t i = 0; i < ent[c].size(); ++i) {
                const uint64_t col = ent[c][i].first >> 20, slot = ent[c][i].first & 0xFFFFF;
                code[toff[t] + i] = (uint32_t)(((col - (uint64_t)c * W) << sb) | slot);
                perm[toff[t] + i] = ent[c][i].second;
            }
        }
    };
    {
        // a host allocation failure inside a worker is reported, not thrown
        // across the thread boundary
        const int nth = std::max(1, std::min<int>(std::min(nblk, 8), (int)std::thread::hardware_concurrency()));
        std::vector<char> failed(nth, 0);
        std::vector<std::thread> pool;
        try {
            for (int h = 0; h < nth; ++h)
                pool.emplace_back([&, h]() {
                    try {
                        for (int b = h; b < nblk; b += nth) lay_block(b);
                    } catch (...) {
                        failed[h] = 1;
                    }
                });
        } catch (...) {
            failed[0] = 1;  // a thread could not be started
        }
        for (auto &th : pool) th.join();
        for (char f : failed)
            if (f) {
                set_error("pp_matrix_create: out of host memory building the column-sorted copy");
                return PP_ENOMEM;
            }
    }
    PP_TRY(dev_alloc(&A->cs_code, (size_t)std::max<int64_t>(ne, 1)));
    PP_TRY(dev_alloc(&A->cs_perm, (size_t)std::max<int64_t>(ne, 1)));
    PP_TRY(dev_alloc(&A->cs_val64, (size_t)std::max<int64_t>(ne, 1)));
    PP_TRY(dev_alloc(&A->cs_val32, (size_t)std::max<int64_t>(ne, 1)));
    PP_TRY(dev_alloc(&A->cs_toff, toff.size()));
    PP_TRY(dev_alloc(&A->cs_tptr, tptr.size()));
    PP_TRY(dev_alloc(&A->cs_part, (size_t)kCsMaxParts * n));
    if ((ne > 0 && (hipMemcpyAsync(A->cs_code, code.data(), sizeof(uint32_t) * ne, hipMemcpyHostToDevice, st) !=
                        hipSuccess ||
                    hipMemcpyAsync(A->cs_perm, perm.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice, st) !=
                        hipSuccess ||
                    launch_sell_values(ne, A->cs_perm, val, A->cs_val64, A->cs_val32, st) != hipSuccess)) ||
        hipMemcpyAsync(A->cs_toff, toff.data(), sizeof(int32_t) * toff.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(A->cs_tptr, tptr.data(), sizeof(uint16_t) * tptr.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("pp_matrix_create: column-sorted upload failed");
        return PP_EDEVICE;
    }
    if (split) {
        PP_TRY(dev_alloc(&A->cs_dperm, (size_t)n));
        PP_TRY(dev_alloc(&A->cs_dg64, (size_t)n));
        PP_TRY(dev_alloc(&A->cs_dg32, (size_t)n));
        if (hipMemcpyAsync(A->cs_dperm, dpos.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
            launch_sell_values(n, A->cs_dperm, val, A->cs_dg64, A->cs_dg32, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("pp_matrix_create: column-sorted upload failed");
            return PP_EDEVICE;
        }
    }
    A->cs_nnz = ne;
    A->cs_nb = nb;
    A->cs_sb = sb;
    A->cs_W = (int)W;
    A->cs_maxe = (int)maxe;
    return PP_OK;
}

// Pattern-coded copy from the value codes (row r's nd codes are
// codes[r G 8 .. r G 8 + nd)): the distinct code tuples of the rows become
// patterns when there are at most 256 of them with at most kMaxPatEntries
// table entries; otherwise the matrix has no pattern-coded copy.
pp_status build_patterns(pp_matrix A, const std::vector<uint8_t> &codes, int nd, const std::vector<double> &tab,
                         hipStream_t st) {
    const int64_t n = A->n;
    const size_t stride = (size_t)((nd + 7) / 8) * 8;
    const int maxpat = std::min(256, kMaxPatEntries / nd);
    std::unordered_map<std::string, int> id_of;
    std::vector<const uint8_t *> pats;
    std::vector<uint32_t> words((size_t)((n + 1023) / 1024) * 256, 0u);
    std::vector<uint8_t> bytes((size_t)((n + 1023) / 1024) * 1024, 0);
    int prev = -1;
    const uint8_t *prevc = nullptr;
    for (int64_t r = 0; r < n; ++r) {
        const uint8_t *c = codes.data() + (size_t)r * stride;
        int id = prev;
        if (!prevc || std::memcmp(c, prevc, nd) != 0) {
            std::string key((const char *)c, nd);
            auto it = id_of.find(key);
            if (it == id_of.end()) {
                if ((int)pats.size() >= maxpat) return PP_OK;
                id = (int)pats.size();
                id_of.emplace(std::move(key), id);
                pats.push_back(c);
            } else {
                id = it->second;
            }
            prev = id;
            prevc = c;
        }
        words[(size_t)(r >> 10) * 256 + (size_t)(r & 255)] |= (uint32_t)id << (8 * ((r >> 8) & 3));
        bytes[(size_t)r] = (uint8_t)id;
    }
    const int npat = (int)pats.size();
    std::vector<double> pt((size_t)npat * nd);
    std::vector<float> pt32(pt.size());
    std::vector<uint8_t> pc(pt.size());
    for (int q = 0; q < npat; ++q)
        for (int d = 0; d < nd; ++d) {
            pc[(size_t)q * nd + d] = pats[q][d];
            pt[(size_t)q * nd + d] = tab[pats[q][d]];
            pt32[(size_t)q * nd + d] = (float)tab[pats[q][d]];
        }
    PP_TRY(dev_alloc(&A->pcodes, pc.size()));
    if (hipMemcpyAsync(A->pcodes, pc.data(), pc.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("pp_matrix_create: pattern-coded upload failed");
        return PP_EDEVICE;
    }
    PP_TRY(dev_alloc(&A->pcode, words.size()));
    PP_TRY(dev_alloc(&A->pbyte, bytes.size()));
    PP_TRY(dev_alloc(&A->ptab64, pt.size()));
    PP_TRY(dev_alloc(&A->ptab32, pt.size()));
    if (hipMemcpyAsync(A->pcode, words.data(), sizeof(uint32_t) * words.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(A->pbyte, bytes.data(), bytes.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(A->ptab64, pt.data(), sizeof(double) * pt.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(A->ptab32, pt32.data(), sizeof(float) * pt.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("pp_matrix_create: pattern-coded upload failed");
        return PP_EDEVICE;
    }
    A->npat = npat;
    return PP_OK;
}

// Value-coded copy of the diagonal format (at most 255 distinct nonzero
// values; code 0 is zero) and the pattern-coded copy built from it, from
// the host values hv and the slot -> entry map dp of the diagonal format.
// Leaves the matrix without the copies (PP_OK) when it does not qualify.
pp_status build_value_codes(pp_matrix A, const int32_t *dp, const std::vector<double> &hv, hipStream_t st) {
    const int64_t n = A->n, nnz = A->nnz;
    const int nd = (int)A->h_doff.size();
    pp_status s;
    std::unordered_map<uint64_t, int> code_of;
    std::vector<double> tab(1, 0.0);
    code_of[0] = 0;
    bool few_values = true;
    for (int64_t q = 0; q < nnz && few_values; ++q) {
        uint64_t bits;
        std::memcpy(&bits, &hv[q], sizeof bits);
        if (code_of.find(bits) == code_of.end()) {
            if (tab.size() >= 256) {
                few_values = false;
                break;
            }
            code_of[bits] = (int)tab.size();
            tab.push_back(hv[q]);
        }
    }
    if (few_values) {
        const int G = (nd + 7) / 8;
        std::vector<uint8_t> codes((size_t)n * G * 8, 0);
        for (int64_t r = 0; r < n; ++r)
            for (int dd = 0; dd < nd; ++dd) {
                const int kk = dp[((r >> 8) * (long)nd + dd) * 256 + (r & 255)];
                if (kk < 0) continue;
                uint64_t bits;
                std::memcpy(&bits, &hv[kk], sizeof bits);
                codes[((size_t)r * G + dd / 8) * 8 + dd % 8] = (uint8_t)code_of[bits];
            }
        std::vector<float> tab32(tab.size());
        for (size_t q = 0; q < tab.size(); ++q) tab32[q] = (float)tab[q];
        std::vector<uint8_t> ec(nnz);
        std::vector<int32_t> rep(tab.size(), -1);
        for (int64_t q = 0; q < nnz; ++q) {
            uint64_t bits;
            std::memcpy(&bits, &hv[q], sizeof bits);
            const int c = code_of[bits];
            ec[q] = (uint8_t)c;
            if (rep[c] < 0) rep[c] = (int32_t)q;
        }
        if ((s = dev_alloc(&A->ecode, ec.size())) != PP_OK ||
            (s = dev_alloc(&A->crep, rep.size())) != PP_OK || (s = dev_alloc(&A->rflag, 1)) != PP_OK)
            return s;
        if (hipMemcpyAsync(A->ecode, ec.data(), ec.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(A->crep, rep.data(), sizeof(int32_t) * rep.size(), hipMemcpyHostToDevice,
                           st) != hipSuccess) {
            set_error("value-coded upload failed");
            return PP_EDEVICE;
        }
        if ((s = dev_alloc(&A->dcode, codes.size())) != PP_OK ||
            (s = dev_alloc(&A->dtab64, tab.size())) != PP_OK ||
            (s = dev_alloc(&A->dtab32, tab.size())) != PP_OK)
            return s;
        if (hipMemcpyAsync(A->dcode, codes.data(), codes.size(), hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(A->dtab64, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice,
                           st) != hipSuccess ||
            hipMemcpyAsync(A->dtab32, tab32.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("value-coded upload failed");
            return PP_EDEVICE;
        }
        A->ntab = (int)tab.size();
        if ((s = build_patterns(A, codes, nd, tab, st)) != PP_OK) return s;
    }
    return PP_OK;
}

// The box geometry of a stencil matrix: diagonals exactly 0, +-1, +-gx
// (and +-gx gy), n = gx gy gz, and no stored entry joining the last point
// of a grid line (or plane) to the first of the next. Leaves box_nd = 0
// when the matrix is not such a stencil.
// A constant-coefficient box stencil: every row's code tuple is the one of
// an interior row with code 0 (the value zero) wherever the neighbour lies
// outside the box, so the interior row's coefficients serve every row of a
// kernel that keeps the points outside the box at zero. The codes stay valid
// when new values keep them (pp_matrix_set_values), so does this.
void detect_box_const(pp_matrix A, hipStream_t st) {
    A->box_pint = -1;
    if (!A->box_nd || !A->pbyte || !A->pcodes || A->npat <= 0) return;
    const long n = A->n;
    const int nd = A->box_nd;
    const long gx = A->box[0], gy = A->box[1], gz = A->box[2];
    if (gx < 3 || gy < 3 || (nd == 7 && gz < 3)) return;
    std::vector<uint8_t> pb((size_t)n), pc((size_t)A->npat * nd);
    if (hipMemcpyAsync(pb.data(), A->pbyte, (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(pc.data(), A->pcodes, pc.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return;
    const long rc = gx / 2 + gx * (gy / 2 + gy * (nd == 7 ? gz / 2 : 0));
    const int pint = pb[(size_t)rc];
    const uint8_t *ci = pc.data() + (size_t)pint * nd;
    for (long r = 0; r < n; ++r) {
        const long x = r % gx, y = (r / gx) % gy, z = r / (gx * gy);
        // neighbours in ascending offset order: (-z) -y -x 0 +x +y (+z)
        bool in[7];
        if (nd == 7) {
            in[0] = z > 0, in[1] = y > 0, in[2] = x > 0, in[3] = true, in[4] = x < gx - 1, in[5] = y < gy - 1,
            in[6] = z < gz - 1;
        } else {
            in[0] = y > 0, in[1] = x > 0, in[2] = true, in[3] = x < gx - 1, in[4] = y < gy - 1;
        }
        const uint8_t *cr = pc.data() + (size_t)pb[(size_t)r] * nd;
        for (int d = 0; d < nd; ++d)
            if (cr[d] != (in[d] ? ci[d] : 0)) return;
    }
    A->box_pint = pint;
}

void detect_box(pp_matrix A, const std::vector<int32_t> &ci) {
    const auto &o = A->h_doff;
    const int nd = (int)o.size();
    const long n = A->n;
    long gx = 0, gy = 0, gz = 0;
    if (nd == 7 && o[0] == -o[6] && o[1] == -o[5] && o[2] == -1 && o[3] == 0 && o[4] == 1 && o[5] >= 2 &&
        o[6] % o[5] == 0 && n % o[6] == 0) {
        gx = o[5];
        gy = o[6] / o[5];
        gz = n / o[6];
    } else if (nd == 5 && o[0] == -o[4] && o[1] == -1 && o[2] == 0 && o[3] == 1 && o[4] >= 2 && n % o[4] == 0) {
        gx = o[4];
        gy = n / o[4];
        gz = 1;
    }
    if (gx < 2 || gy < 2 || gz < 1) return;
    const auto &rp = A->h_rowptr;
    for (long r = 0; r < n; ++r) {
        const long x = r % gx, y = (r / gx) % gy;
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const long off = (long)ci[k] - r;
            if ((off == 1 && x == gx - 1) || (off == -1 && x == 0) || (nd == 7 && off == gx && y == gy - 1) ||
                (nd == 7 && off == -gx && y == 0))
                return;
        }
    }
    A->box[0] = (int)gx;
    A->box[1] = (int)gy;
    A->box[2] = (int)gz;
    A->box_nd = nd;
}

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
    std::vector<int32_t> ci(nnz);
    if (nnz > 0) {
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
    // row-tile plans of the two tile variants
    std::vector<int4> t8, t16;
    // capacities leave room for the 16-byte alignment of the vector-load variants
    build_tiles(rp.data(), (int)n, 256, 256 * 8 - 4, t8);
    build_tiles(rp.data(), (int)n, 512, 256 * 16 - 4, t16);
    A->ntile8 = (int)t8.size();
    A->ntile16 = (int)t16.size();
    // persistent kernel: the largest co-resident grid over the three
    // precisions, and a tile plan balanced so that every workgroup owns about
    // the same number of stored entries
    {
        int g0 = 0, g1 = 0, g2 = 0;
        if (persist_max_grid(0, &g0) != hipSuccess || persist_max_grid(1, &g1) != hipSuccess ||
            persist_max_grid(2, &g2) != hipSuccess) {
            set_error("pp_matrix_create: occupancy query failed");
            return fail(PP_EDEVICE);
        }
        A->pgrid = std::max(0, std::min(g0, std::min(g1, g2)));
    }
    std::vector<int4> tP;
    if (A->pgrid > 0) {
        const long G = A->pgrid;
        const long per_wg = std::max<long>(1, (nnz + G - 1) / G);
        const long k = std::max<long>(1, (per_wg + (256 * 8 - 4) - 1) / (256 * 8 - 4));
        const long cap = std::max<long>(1, (per_wg + k - 1) / k);
        build_tiles(rp.data(), (int)n, 256, (int)std::min<long>(cap, 256 * 8 - 4), tP);
    }
    A->ntileP = (int)tP.size();
    A->nblk_dot = dot_blocks(A->n);
    A->nblk_upd = (A->n + 255) / 256;
    A->nblk_ud = update_dots_blocks(A->n);
    pp_status s;
    if ((s = dev_alloc(&A->tile8, t8.size())) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->tile16, t16.size())) != PP_OK) return fail(s);
    if (!tP.empty() && (s = dev_alloc(&A->tileP, tP.size())) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->bar, 1)) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->err, 1)) != PP_OK) return fail(s);
    if (hipHostMalloc((void **)&A->errpin, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        A->errpin = nullptr;
        set_error("hipHostMalloc failed");
        return fail(PP_ENOMEM);
    }
    *A->errpin = 0;
    if ((s = dev_alloc(&A->val32, (size_t)std::max<int64_t>(nnz, 1))) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->npart, (size_t)A->nblk_upd)) != PP_OK) return fail(s);
    if ((s = dev_alloc(&A->r64, (size_t)2 * A->n)) != PP_OK) return fail(s);
    A->t64 = A->r64 + A->n;
    if ((s = A->ensure_red(64)) != PP_OK) return fail(s);
    if (hipMemcpyAsync(A->tile8, t8.data(), sizeof(int4) * t8.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(A->tile16, t16.data(), sizeof(int4) * t16.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        (!tP.empty() &&
         hipMemcpyAsync(A->tileP, tP.data(), sizeof(int4) * tP.size(), hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemsetAsync(A->bar, 0, sizeof(unsigned long long), st) != hipSuccess ||
        hipMemsetAsync(A->err, 0, sizeof(int), st) != hipSuccess ||
        launch_val_to_f32((int)nnz, val, A->val32, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        set_error("pp_matrix_create: device upload failed");
        return fail(PP_EDEVICE);
    }
    // Sliced-ELL copy (64-row slices, entries of a slice stored column by
    // column) when the padding stays below a quarter of the entries.
    {
        const int ns = (int)((n + 63) / 64);
        std::vector<int32_t> sp(ns + 1, 0);
        long tot = 0;
        for (int w = 0; w < ns; ++w) {
            int width = 0;
            for (int r = w * 64; r < std::min<int64_t>((int64_t)w * 64 + 64, n); ++r) width = std::max(width, rp[r + 1] - rp[r]);
            tot += 64L * width;
            sp[w + 1] = (int32_t)std::min<long>(tot, (1L << 31) - 1);
        }
        if (nnz > 0 && tot <= nnz + nnz / 4 + 64L * 8 && tot < (1L << 31)) {
            std::vector<int32_t> scol(tot, 0), sperm(tot, -1);
            for (int w = 0; w < ns; ++w) {
                const int width = (sp[w + 1] - sp[w]) / 64;
                for (int j = 0; j < 64; ++j) {
                    const long r = (long)w * 64 + j;
                    const int len = r < n ? rp[r + 1] - rp[r] : 0;
                    for (int k = 0; k < width; ++k) {
                        const long o = sp[w] + (long)k * 64 + j;
                        if (k < len) {
                            scol[o] = ci[rp[r] + k];
                            sperm[o] = rp[r] + k;
                        } else {
                            scol[o] = r < n ? (int32_t)r : 0;  // padding: a valid index with value 0
                        }
                    }
                }
            }
            if ((s = dev_alloc(&A->sptr, sp.size())) != PP_OK || (s = dev_alloc(&A->scol, (size_t)tot)) != PP_OK ||
                (s = dev_alloc(&A->sperm, (size_t)tot)) != PP_OK || (s = dev_alloc(&A->sval64, (size_t)tot)) != PP_OK ||
                (s = dev_alloc(&A->sval32, (size_t)tot)) != PP_OK)
                return fail(s);
            if (hipMemcpyAsync(A->sptr, sp.data(), sizeof(int32_t) * sp.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(A->scol, scol.data(), sizeof(int32_t) * tot, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(A->sperm, sperm.data(), sizeof(int32_t) * tot, hipMemcpyHostToDevice, st) != hipSuccess ||
                launch_sell_values(tot, A->sperm, val, A->sval64, A->sval32, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                set_error("pp_matrix_create: sliced-ELL upload failed");
                return fail(PP_EDEVICE);
            }
            A->nslices = ns;
            A->npad = tot;
            // 16-bit column offsets when every entry is within 32767 of its row
            bool fits = true;
            std::vector<int16_t> sdel(tot);
            for (int w = 0; w < ns && fits; ++w)
                for (long o = sp[w]; o < sp[w + 1]; ++o) {
                    const long row = (long)w * 64 + (o - sp[w]) % 64;
                    // rows past n are padding (column 0, value 0): offset 0 from base 0
                    const long dlt = row < n ? (long)scol[o] - row : 0;
                    if (dlt < -32768 || dlt > 32767) {
                        fits = false;
                        break;
                    }
                    sdel[o] = (int16_t)dlt;
                }
            if (fits) {
                if ((s = dev_alloc(&A->sdel, (size_t)tot)) != PP_OK) return fail(s);
                if (hipMemcpyAsync(A->sdel, sdel.data(), sizeof(int16_t) * tot, hipMemcpyHostToDevice, st) !=
                        hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess) {
                    set_error("pp_matrix_create: offset upload failed");
                    return fail(PP_EDEVICE);
                }
            }
        }
    }
    // diagonal format when the entries lie on at most kMaxDiag diagonals and
    // the padding stays under a quarter of nnz
    if (nnz > 0) {
        std::vector<int> offs;
        bool few = true;
        for (int64_t r = 0; r < n && few; ++r)
            for (int k = rp[r]; k < rp[r + 1]; ++k) {
                const int off = ci[k] - (int)r;
                if (std::find(offs.begin(), offs.end(), off) == offs.end()) {
                    offs.push_back(off);
                    if ((int)offs.size() > kMaxDiag) {
                        few = false;
                        break;
                    }
                }
            }
        const long nblk = ((long)n + 255) / 256;
        const long slots = (long)offs.size() * nblk * 256;
        if (few && slots <= (long)nnz + nnz / 4 + 64 && slots < (1L << 31)) {
            std::sort(offs.begin(), offs.end());
            std::vector<int32_t> dp(slots, -1);
            for (int64_t r = 0; r < n; ++r)
                for (int k = rp[r]; k < rp[r + 1]; ++k) {
                    const int d = (int)(std::lower_bound(offs.begin(), offs.end(), ci[k] - (int)r) - offs.begin());
                    dp[((r >> 8) * (long)offs.size() + d) * 256 + (r & 255)] = k;  // a repeat keeps its last entry
                }
            // repeated entries of one (row, column) cannot share a slot: no diagonal format then
            long used = 0;
            for (long q = 0; q < slots; ++q) used += dp[q] >= 0;
            if (used == nnz) {
                if ((s = dev_alloc(&A->dval64, (size_t)slots)) != PP_OK ||
                    (s = dev_alloc(&A->dval32, (size_t)slots)) != PP_OK ||
                    (s = dev_alloc(&A->dperm, (size_t)slots)) != PP_OK)
                    return fail(s);
                if (hipMemcpyAsync(A->dperm, dp.data(), sizeof(int32_t) * slots, hipMemcpyHostToDevice, st) !=
                        hipSuccess ||
                    launch_sell_values(slots, A->dperm, val, A->dval64, A->dval32, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess) {
                    set_error("pp_matrix_create: diagonal-format upload failed");
                    return fail(PP_EDEVICE);
                }
                A->h_doff = offs;
                // value-coded copy (and the pattern-coded one built from it)
                const int nd = (int)offs.size();
                const bool nd_ok = nd <= 9 || nd == 13 || nd == 19 || nd == 27;
                std::vector<double> hv(nnz);
                if (nd_ok && hipMemcpyAsync(hv.data(), val, sizeof(double) * nnz, hipMemcpyDeviceToHost, st) ==
                                 hipSuccess &&
                    hipStreamSynchronize(st) == hipSuccess)
                    if ((s = build_value_codes(A, dp.data(), hv, st)) != PP_OK) return fail(s);
                if (A->pbyte) detect_box(A, ci);
                detect_box_const(A, st);
            }
        }
    }
    // column-banded copies for large matrices without a diagonal-format copy
    // (their gathers reach across the whole input)
    if (nnz > 0 && n >= 4096 && A->h_doff.empty()) {
        if ((s = build_bands(A, rp, ci, val, 0, 2, st)) != PP_OK) return fail(s);
        if ((s = build_bands(A, rp, ci, val, 1, 4, st)) != PP_OK) return fail(s);
        if ((s = build_csort(A, rp, ci, val, st)) != PP_OK) return fail(s);
    }
    {
        // tuning program of the persistent kernel: 8 sparse products P0 -> P1 -> P0 ...
        std::vector<PStep> h(8);
        for (int i = 0; i < 8; ++i) {
            std::memset(&h[i], 0, sizeof(PStep));
            h[i].spmv = 1;
            h[i].in = (i % 2 == 0) ? B_P0 : B_P1;
            h[i].out = (i % 2 == 0) ? B_P1 : B_P0;
            h[i].aux = h[i].acc = -1;
            h[i].a0 = 1.0;
        }
        if ((s = upload_steps(h, &A->tune_steps, st)) != PP_OK) return fail(s);
    }
    *out = A;
    return PP_OK;
}

}  // extern "C"

namespace {

// Point the handle at new FP64 values and refresh the copies derived from them.
pp_status refresh_values(pp_matrix A, const double *val, hipStream_t st) {
    A->val = val;
    HIP_TRY(launch_val_to_f32(A->nnz, val, A->val32, st));
    if (A->nslices > 0) HIP_TRY(launch_sell_values(A->npad, A->sperm, val, A->sval64, A->sval32, st));
    if (!A->h_doff.empty())
        HIP_TRY(launch_sell_values((long)A->h_doff.size() * (((long)A->n + 255) / 256) * 256, A->dperm, val,
                                   A->dval64, A->dval32, st));
    for (int c = 0; c < 2; ++c)
        if (A->bandK[c] > 0) HIP_TRY(launch_sell_values(A->bnnz[c], A->bperm[c], val, A->bval64[c], A->bval32[c], st));
    if (A->cs_nb > 0) {
        if (A->cs_nnz > 0) HIP_TRY(launch_sell_values(A->cs_nnz, A->cs_perm, val, A->cs_val64, A->cs_val32, st));
        if (A->cs_dperm) HIP_TRY(launch_sell_values(A->n, A->cs_dperm, val, A->cs_dg64, A->cs_dg32, st));
    }
    if (A->dcode) {
        // the codes stay when every entry still equals its code's new value
        // (a constant-coefficient stencil with new coefficients); else drop
        // them, and a tuned pick of them
        HIP_TRY(launch_recode(A->nnz, val, A->ecode, A->crep, A->ntab, A->dtab64, A->dtab32,
                              A->pcode ? A->npat * (int)A->h_doff.size() : 0, A->pcodes, A->ptab64, A->ptab32,
                              A->rflag, st));
        int *fl = reinterpret_cast<int *>(A->hpin);
        HIP_TRY(hipMemcpyAsync(fl, A->rflag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (*fl) {
            dev_free(A->dcode);
            dev_free(A->dtab64);
            dev_free(A->dtab32);
            dev_free(A->ecode);
            dev_free(A->crep);
            dev_free(A->pcodes);
            dev_free(A->rflag);
            dev_free(A->pcode);
            dev_free(A->pbyte);
            dev_free(A->ptab64);
            dev_free(A->ptab32);
            A->ntab = 0;
            A->npat = 0;
            A->box_pint = -1;
            for (int p = 0; p < 3; ++p)
                if (A->variant[p] == CV_DIAC || A->variant[p] == CV_DIAP || A->variant[p] == CV_DIAPV ||
                    A->variant[p] == CV_BOX) {
                    A->variant[p] = CV_TILE8;
                    A->tuned[p] = 0;
                }
            // once per handle, code the new values afresh (classes change
            // when, e.g., a coefficient that was zero no longer is; later
            // values of the same classes then keep the codes)
            if (!A->recoded) {
                A->recoded = true;
                const long slots = (long)A->h_doff.size() * (((long)A->n + 255) / 256) * 256;
                std::vector<int32_t> dp(slots);
                std::vector<double> hv(A->nnz);
                HIP_TRY(hipMemcpyAsync(dp.data(), A->dperm, sizeof(int32_t) * slots, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(hv.data(), val, sizeof(double) * A->nnz, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                PP_TRY(build_value_codes(A, dp.data(), hv, st));
                detect_box_const(A, st);
            }
        }
    }
    return PP_OK;
}

// Values of A diag(s) from the caller's values (Jacobi: s from their diagonal).
pp_status apply_scaling(pp_matrix A, hipStream_t st, const char *who) {
    if (A->scale_mode == 1) {
        int *bad = nullptr;
        PP_TRY(dev_alloc(&bad, 1));
        struct Free {
            int *p;
            ~Free() { dev_free(p); }
        } fb{bad};
        int hbad = 0;
        HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), st));
        HIP_TRY(launch_jacobi(A->n, A->rowptr, A->colind, A->user_val, A->scale, bad, st));
        HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (hbad) {
            set_error(std::string(who) + ": a diagonal entry is missing or zero (Jacobi scaling)");
            return PP_ESINGULAR;
        }
    }
    HIP_TRY(launch_scale_cols(A->nnz, A->colind, A->user_val, A->scale, A->val_own, st));
    return refresh_values(A, A->val_own, st);
}

// Back to the caller's unscaled values (after a failed scaling).
void drop_scaling(pp_matrix A, hipStream_t st) {
    A->scale_mode = 0;
    (void)refresh_values(A, A->user_val, st);
    (void)hipStreamSynchronize(st);
    dev_free(A->val_own);
    dev_free(A->scale);
    A->val_own = nullptr;
    A->scale = nullptr;
}

}  // namespace

namespace {

// Inverse of the m x m matrix a (row-major, overwritten) into inv (row
// stride ld) by Gauss-Jordan elimination with partial pivoting; false if a
// pivot is exactly zero.
bool invert_block(int m, std::vector<double> &a, double *inv, int ld) {
    std::vector<double> b((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) b[(size_t)i * m + i] = 1.0;
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(a[(size_t)r * m + c]) > std::fabs(a[(size_t)p * m + c])) p = r;
        const double piv = a[(size_t)p * m + c];
        if (piv == 0.0) return false;
        if (p != c)
            for (int k = 0; k < m; ++k) {
                std::swap(a[(size_t)p * m + k], a[(size_t)c * m + k]);
                std::swap(b[(size_t)p * m + k], b[(size_t)c * m + k]);
            }
        for (int k = 0; k < m; ++k) {
            a[(size_t)c * m + k] /= piv;
            b[(size_t)c * m + k] /= piv;
        }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = a[(size_t)r * m + c];
            if (f == 0.0) continue;
            for (int k = 0; k < m; ++k) {
                a[(size_t)r * m + k] -= f * a[(size_t)c * m + k];
                b[(size_t)r * m + k] -= f * b[(size_t)c * m + k];
            }
        }
    }
    for (int r = 0; r < m; ++r)
        for (int k = 0; k < m; ++k) inv[(size_t)r * ld + k] = b[(size_t)r * m + k];
    return true;
}

// B = A M^{-1} for the block-Jacobi M of A's current values (blocks of bs
// rows): M^{-1}'s blocks into minv (stride bs), B's CSR into brp/bci/bv
// (built only when bci is not null; nnz_b always). Row i of B: for each
// block J its columns touch, sum_j a_ij (M^{-1})_{j, J bs + c} over the
// entries j of that block, in column order, for every column c of J.
pp_status block_jacobi_build(pp_matrix A, int bs, hipStream_t st, int64_t *nnz_b, std::vector<double> &minv,
                             std::vector<int32_t> *brp, std::vector<int32_t> *bci, std::vector<double> *bv) {
    if (A->scale_mode != 0 || A->rbs > 0) {
        set_error("block-Jacobi: the handle already has a right preconditioner");
        return PP_EINVAL;
    }
    const int64_t n = A->n, nnz = A->nnz;
    const int64_t nb = (n + bs - 1) / bs;
    std::vector<int32_t> ci(nnz);
    std::vector<double> hv(nnz);
    if (nnz) {
        HIP_TRY(hipMemcpyAsync(ci.data(), A->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hv.data(), A->val, sizeof(double) * nnz, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    const auto &rp = A->h_rowptr;
    minv.assign((size_t)nb * bs * bs, 0.0);
    std::vector<double> d;
    for (int64_t k = 0; k < nb; ++k) {
        const int64_t r0 = k * bs;
        const int m = (int)std::min<int64_t>(bs, n - r0);
        d.assign((size_t)m * m, 0.0);
        for (int64_t r = r0; r < r0 + m; ++r)
            for (int e = rp[r]; e < rp[r + 1]; ++e)
                if (ci[e] >= r0 && ci[e] < r0 + m) d[(size_t)(r - r0) * m + (ci[e] - r0)] += hv[e];
        if (!invert_block(m, d, minv.data() + (size_t)k * bs * bs, bs)) {
            set_error("block-Jacobi: a diagonal block is singular");
            return PP_ESINGULAR;
        }
    }
    int64_t tot = 0;
    std::vector<std::pair<int32_t, double>> row;
    std::vector<double> acc(bs);
    if (brp) brp->assign((size_t)n + 1, 0);
    if (bci) {
        bci->clear();
        bv->clear();
    }
    for (int64_t i = 0; i < n; ++i) {
        row.clear();
        for (int e = rp[i]; e < rp[i + 1]; ++e) row.emplace_back(ci[e], hv[e]);
        std::stable_sort(row.begin(), row.end(),
                         [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                             return a.first < b.first;
                         });
        for (size_t q = 0; q < row.size();) {
            const int64_t J = row[q].first / bs, c0 = J * bs;
            const int mJ = (int)std::min<int64_t>(bs, n - c0);
            std::fill(acc.begin(), acc.end(), 0.0);
            for (; q < row.size() && row[q].first / bs == J; ++q) {
                const double *mr = minv.data() + (size_t)J * bs * bs + (size_t)(row[q].first - c0) * bs;
                for (int c = 0; c < mJ; ++c) acc[c] += row[q].second * mr[c];
            }
            tot += mJ;
            if (bci)
                for (int c = 0; c < mJ; ++c) {
                    bci->push_back((int32_t)(c0 + c));
                    bv->push_back(acc[c]);
                }
        }
        if (brp) (*brp)[(size_t)i + 1] = (int32_t)tot;
        if (tot >= (1LL << 31)) {
            set_error("block-Jacobi: B = A M^{-1} has too many entries");
            return PP_EINVAL;
        }
    }
    *nnz_b = tot;
    return PP_OK;
}

}  // namespace

extern "C" {

pp_status pp_matrix_set_values(pp_matrix A, const double *val, void *stream) {
    if (!A || (!val && A->nnz > 0)) {
        set_error("pp_matrix_set_values: bad argument");
        return PP_EINVAL;
    }
    if (A->scale_mode != 0) {
        A->user_val = val;
        const pp_status r = apply_scaling(A, S(stream), "pp_matrix_set_values");
        if (r != PP_OK) drop_scaling(A, S(stream));
        return r;
    }
    return refresh_values(A, val, S(stream));
}

pp_status pp_matrix_right_scale(pp_matrix A, const double *s, void *stream) {
    if (!A || A->nnz == 0) {
        set_error("pp_matrix_right_scale: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    if (A->scale_mode == 0) {
        A->user_val = A->val;
        PP_TRY(dev_alloc(&A->val_own, (size_t)A->nnz));
        PP_TRY(dev_alloc(&A->scale, (size_t)A->n));
    }
    if (s) {
        HIP_TRY(hipMemcpyAsync(A->scale, s, sizeof(double) * A->n, hipMemcpyDeviceToDevice, st));
        A->scale_mode = 2;
    } else {
        A->scale_mode = 1;
    }
    const pp_status r = apply_scaling(A, st, "pp_matrix_right_scale");
    if (r != PP_OK) drop_scaling(A, st);
    return r;
}

pp_status pp_matrix_scale(pp_matrix A, double *s, void *stream) {
    if (!A || !s) {
        set_error("pp_matrix_scale: bad argument");
        return PP_EINVAL;
    }
    if (A->scale_mode == 0) {
        set_error("pp_matrix_scale: the matrix has no right scaling");
        return PP_EINVAL;
    }
    HIP_TRY(hipMemcpyAsync(s, A->scale, sizeof(double) * A->n, hipMemcpyDeviceToDevice, S(stream)));
    return PP_OK;
}

pp_status pp_block_jacobi_nnz(pp_matrix A, int bs, void *stream, int64_t *nnz_b) {
    if (!A || !nnz_b || bs < 1 || bs > kMaxRightBlock) {
        set_error("pp_block_jacobi_nnz: bad argument");
        return PP_EINVAL;
    }
    std::vector<double> minv;
    try {
        return block_jacobi_build(A, bs, S(stream), nnz_b, minv, nullptr, nullptr, nullptr);
    } catch (const std::bad_alloc &) {
        set_error("pp_block_jacobi_nnz: out of host memory");
        return PP_ENOMEM;
    }
}

pp_status pp_block_jacobi(pp_matrix A, int bs, int32_t *rowptr_b, int32_t *colind_b, double *val_b, double *minv,
                          void *stream) {
    if (!A || !rowptr_b || !colind_b || !val_b || !minv || bs < 1 || bs > kMaxRightBlock) {
        set_error("pp_block_jacobi: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    int64_t nb = 0;
    std::vector<double> mv, bv;
    std::vector<int32_t> brp, bci;
    try {
        PP_TRY(block_jacobi_build(A, bs, st, &nb, mv, &brp, &bci, &bv));
    } catch (const std::bad_alloc &) {
        set_error("pp_block_jacobi: out of host memory");
        return PP_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(rowptr_b, brp.data(), sizeof(int32_t) * brp.size(), hipMemcpyHostToDevice, st));
    if (nb) {
        HIP_TRY(hipMemcpyAsync(colind_b, bci.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(val_b, bv.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipMemcpyAsync(minv, mv.data(), sizeof(double) * mv.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PP_OK;
}

pp_status pp_matrix_right_blocks(pp_matrix B, int bs, const double *minv, void *stream) {
    if (!B || !minv || bs < 1 || bs > kMaxRightBlock) {
        set_error("pp_matrix_right_blocks: bad argument");
        return PP_EINVAL;
    }
    const size_t len = (size_t)((B->n + bs - 1) / bs) * bs * bs;
    dev_free(B->rminv);
    B->rbs = 0;
    PP_TRY(dev_alloc(&B->rminv, len));
    HIP_TRY(hipMemcpyAsync(B->rminv, minv, sizeof(double) * len, hipMemcpyDeviceToDevice, S(stream)));
    B->rbs = bs;
    return PP_OK;
}

void pp_matrix_destroy(pp_matrix A) { delete A; }

pp_status pp_matrix_tune(pp_matrix A, int prec, void *stream, int *variant, int *remap, double *us_per_launch) {
    if (!A || !valid_prec(prec)) {
        set_error("pp_matrix_tune: bad argument");
        return PP_EINVAL;
    }
    PP_TRY(tune_chain(A, prec, S(stream)));
    if (variant) *variant = A->persist[prec] ? (int)CV_PERSIST : A->variant[prec];
    if (remap) *remap = A->persist[prec] ? A->premap[prec] : A->remap[prec];
    if (us_per_launch) *us_per_launch = A->tuned_us[prec];
    return PP_OK;
}

pp_status pp_matrix_set_variant(pp_matrix A, int prec, int variant, int remap) {
    if (!A || !valid_prec(prec) || variant < 0 || variant >= CV_COUNT || (remap != 0 && remap != 1)) {
        set_error("pp_matrix_set_variant: bad argument");
        return PP_EINVAL;
    }
    if (variant == CV_PERSIST) {
        if (A->pgrid <= 0) {
            set_error("pp_matrix_set_variant: persistent kernel unavailable");
            return PP_EINVAL;
        }
        A->persist[prec] = 1;
        A->premap[prec] = remap;
    } else {
        if (((variant == CV_SELL || variant == CV_SELLT || variant == CV_SELL2 || variant == CV_SELL4) && A->nslices == 0) ||
            ((variant == CV_SELLD || variant == CV_SELLD4) && !A->sdel)) {
            set_error("pp_matrix_set_variant: no sliced-ELL copy for this matrix (too much padding)");
            return PP_EINVAL;
        }
        if ((variant == CV_DIA || variant == CV_DIA4) && A->h_doff.empty()) {
            set_error("pp_matrix_set_variant: no diagonal-format copy for this matrix (too many diagonals)");
            return PP_EINVAL;
        }
        if (variant == CV_DIAC && !A->dcode) {
            set_error("pp_matrix_set_variant: no value-coded diagonal copy (too many diagonals or distinct values, "
                      "or the values changed)");
            return PP_EINVAL;
        }
        if ((variant == CV_BAND2 && A->bandK[0] == 0) || (variant == CV_BAND4 && A->bandK[1] == 0)) {
            set_error("pp_matrix_set_variant: no column-banded copy (built only for matrices of at least 4096 rows "
                      "whose entries lie far from the diagonal)");
            return PP_EINVAL;
        }
        if ((variant == CV_CSORT4 || variant == CV_CSORT2) && A->cs_nb == 0) {
            set_error("pp_matrix_set_variant: no column-sorted copy (built only for matrices of at least 4096 rows "
                      "whose entries lie far from the diagonal, when every tile fits)");
            return PP_EINVAL;
        }
        if ((variant == CV_DIAP && !A->pcode) || (variant == CV_DIAPV && !A->pbyte)) {
            set_error("pp_matrix_set_variant: no pattern-coded diagonal copy (no value-coded copy, too many "
                      "distinct rows, or the values changed)");
            return PP_EINVAL;
        }
        if (variant == CV_BOX && !box_step_ok(A->dev())) {
            set_error("pp_matrix_set_variant: the box kernel needs a constant-coefficient 5- or 7-point box stencil "
                      "whose grid lines hold a multiple of 4 points");
            return PP_EINVAL;
        }
        if (variant == CV_TILEB8) PP_TRY(build_round_plan(A, prec, 8, &A->tileB8[prec], &A->ntileB8[prec], 0));
        if (variant == CV_TILEB16) PP_TRY(build_round_plan(A, prec, 16, &A->tileB16[prec], &A->ntileB16[prec], 0));
        A->persist[prec] = 0;
        A->variant[prec] = variant;
        A->remap[prec] = remap;
    }
    A->tuned[prec] = 1;
    A->tuned_us[prec] = 0.0;
    A->fuse[prec] = 0;  // the forced variant runs every step
    A->march[prec] = 0;
    A->march_all[prec] = 0;
    A->march_tile[prec] = 0;
    A->pair_tile[prec] = 0;
    return PP_OK;
}

pp_status pp_matrix_set_pair_steps(pp_matrix A, int prec, int mode) {
    if (!A || !valid_prec(prec) || (mode != 0 && mode != 1)) {
        set_error("pp_matrix_set_pair_steps: bad argument");
        return PP_EINVAL;
    }
    if (mode == 1 && (!A->box_nd || !A->pbyte || prec == PP_BF16S)) {
        set_error("pp_matrix_set_pair_steps: two steps per launch need a 5- or 7-point box stencil with a "
                  "pattern-coded copy, and FP64 or FP32 vectors");
        return PP_EINVAL;
    }
    if (!A->tuned[prec]) {
        set_error("pp_matrix_set_pair_steps: tune or set the precision's variant first");
        return PP_EINVAL;
    }
    A->fuse[prec] = mode;
    return PP_OK;
}

pp_status pp_matrix_set_march(pp_matrix A, int prec, int steps, int cz, int depth) {
    if (!A || !valid_prec(prec) || steps < 0 || steps == 1 || steps > kMarchMax || cz < 0 || depth < 0 ||
        depth > 3) {
        set_error("pp_matrix_set_march: bad argument");
        return PP_EINVAL;
    }
    if (steps >= 2 && (!A->box_nd || !A->pbyte || prec == PP_BF16S)) {
        set_error("pp_matrix_set_march: several steps per launch need a 5- or 7-point box stencil with a "
                  "pattern-coded copy, and FP64 or FP32 vectors");
        return PP_EINVAL;
    }
    if (!A->tuned[prec] || A->persist[prec]) {
        set_error("pp_matrix_set_march: tune or set a single-launch variant for this precision first");
        return PP_EINVAL;
    }
    A->march[prec] = steps;
    A->march_all[prec] = steps >= 2;
    A->march_tile[prec] = 0;
    const int c = cz > 0 ? cz : march_default_cz(A->dev(), 1024);
    for (int g = 2; g <= kMarchMax; ++g) {
        A->march_cz[prec][g] = c;
        A->march_depth[prec][g] = depth > 0 ? depth : 1;
    }
    return PP_OK;
}

pp_status pp_matrix_set_march_shape(pp_matrix A, int prec, int shape) {
    if (!A || !valid_prec(prec) || (shape != 0 && shape != 1)) {
        set_error("pp_matrix_set_march_shape: bad argument");
        return PP_EINVAL;
    }
    if (!A->tuned[prec] || A->persist[prec]) {
        set_error("pp_matrix_set_march_shape: tune or set a single-launch variant for this precision first");
        return PP_EINVAL;
    }
    if (shape == 1 && !box_tile_ok(A->dev(), prec)) {
        set_error("pp_matrix_set_march_shape: whole-line tiles need a constant-coefficient 7-point box stencil "
                  "whose grid lines hold 64, 128 or 256 points, and FP64 or FP32 vectors");
        return PP_EINVAL;
    }
    A->march_tile[prec] = shape;
    A->pair_tile[prec] = shape;
    if (shape == 1) {
        A->march[prec] = 2;
        A->march_all[prec] = 1;
        A->fuse[prec] = 1;  // the pairs of p chains too
    }
    return PP_OK;
}

pp_status pp_matrix_march_shape(pp_matrix A, int prec, int *shape) {
    if (!A || !valid_prec(prec) || !shape) {
        set_error("pp_matrix_march_shape: bad argument");
        return PP_EINVAL;
    }
    *shape = A->march[prec] >= 2 && A->march_tile[prec] ? 1 : 0;
    return PP_OK;
}

pp_status pp_matrix_march(pp_matrix A, int prec, int *steps, int *cz, double *us, int *constant) {
    if (!A || !valid_prec(prec) || !steps) {
        set_error("pp_matrix_march: bad argument");
        return PP_EINVAL;
    }
    const int g = A->box_nd && A->pbyte && prec != PP_BF16S ? A->march[prec] : 0;
    *steps = g;
    if (cz) *cz = g >= 2 ? A->march_cz[prec][g] : 0;
    if (us) *us = g >= 2 ? A->march_us[prec][g] : 0.0;
    if (constant) *constant = A->box_nd && A->pbyte && A->box_pint >= 0 ? 1 : 0;
    return PP_OK;
}

pp_status pp_matrix_pair_steps(pp_matrix A, int prec, int *mode, int *box, double *us_pair) {
    if (!A || !valid_prec(prec) || !mode) {
        set_error("pp_matrix_pair_steps: bad argument");
        return PP_EINVAL;
    }
    *mode = A->fuse[prec] && A->box_nd && A->pbyte ? 1 : 0;
    if (box)
        for (int k = 0; k < 3; ++k) box[k] = A->box_nd ? A->box[k] : 0;
    if (us_pair) *us_pair = A->pair_us[prec];
    return PP_OK;
}

pp_status pp_matrix_variant(pp_matrix A, int prec, int *variant, int *remap, double *us_per_launch) {
    if (!A || !valid_prec(prec) || !variant) {
        set_error("pp_matrix_variant: bad argument");
        return PP_EINVAL;
    }
    const bool per = A->tuned[prec] && A->persist[prec];
    *variant = !A->tuned[prec] ? -1 : (per ? (int)CV_PERSIST : A->variant[prec]);
    if (remap) *remap = per ? A->premap[prec] : A->remap[prec];
    if (us_per_launch) *us_per_launch = A->tuned[prec] ? A->tuned_us[prec] : 0.0;
    return PP_OK;
}

const char *pp_chain_variant_name(int variant) { return chain_variant_name(variant); }

pp_status pp_matrix_transpose(pp_matrix A, int32_t *rowptr_t, int32_t *colind_t, int32_t *perm, void *stream) {
    if (!A || !rowptr_t || (A->nnz > 0 && (!colind_t || !perm))) {
        set_error("pp_matrix_transpose: bad argument");
        return PP_EINVAL;
    }
    if (A->rbs > 0) {
        set_error("pp_matrix_transpose: the handle has a block-Jacobi right preconditioner");
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

}  // extern "C"

namespace {

// One GMRES(d) cycle on A from v0 in FP64 (Algorithm 4 step 1a). Hbar
// receives the (d+1) x d Hessenberg matrix (column-major, leading dimension
// d+1), k the Krylov dimension reached (k < d after a breakdown) and dots
// the inner products used.
//
// The orthogonalisation is classical Gram-Schmidt with the second pass and
// the normalisation delayed by one step. The pending vector u (projected
// once against v_0..v_{j-1}) goes into the product w = op(u) before it is
// final. Then one pass of dot products ([V_j u w]^T [u w]), one workgroup of
// coefficient algebra, and one update pass finish v_j = (u - V_j a)/rho and
// form the next pending vector from w through the Arnoldi relation
// A V_j = V_{j+1} Hbar: two sweeps over the basis per step instead of
// three. A last dot pass finishes column d-1.
// basis: the precision the Krylov vectors are stored in (0 binary64, 1
// binary32; dot products, norms and the Hessenberg in FP64 either way).
pp_status setup_arnoldi(pp_matrix A, const double *v0, int d, hipStream_t st, std::vector<double> &Hbar, int &k,
                        bool &brk, int64_t &dots, const char *who, pp_poly op = nullptr, int basis = 0) {
    if (basis != 0 && basis != 1) {
        set_error(std::string(who) + ": basis precision must be FP64 or FP32");
        return PP_EINVAL;
    }
    PP_TRY(A->ensure_ws(basis, d));
    PP_TRY(A->ensure_red(2 * d + 4));
    const Workspace &ws = A->ws[basis];
    const int n = A->n;
    void *u = ws.D, *w = ws.ACC;
    double v0n = 0.0;
    PP_TRY(dev_norm(A, 0, v0, &v0n, st));
    if (!(v0n > 0.0) || !std::isfinite(v0n)) {
        set_error(std::string(who) + ": start vector is zero or not finite");
        return PP_EINVAL;
    }
    if (basis == 0)
        HIP_TRY(hipMemcpyAsync(u, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    else
        HIP_TRY(launch_convert(0, basis, n, v0, u, st));
    // All steps are queued without a host round trip: the Hessenberg columns
    // stay in device memory and the host looks for a breakdown once at the
    // end (columns after a breakdown are discarded).
    const int ld = d + 1;
    double *Hdev = nullptr;
    PP_TRY(dev_alloc(&Hdev, (size_t)ld * d));
    struct Free {
        double *p;
        ~Free() { dev_free(p); }
    } free_h{Hdev};
    HIP_TRY(hipMemsetAsync(Hdev, 0, sizeof(double) * ld * d, st));
    double *dd = A->h1();    // reduced dots, then g (3 d + 6 values over h1, h2, H)
    double *pend = A->z();   // first-pass coefficients of the pending column
    double *coef = A->inv(); // {1/rho, g_j}
    for (int j = 0; j <= d; ++j) {
        const bool last = j == d;
        if (!last) {
            // the operator: A, or phi1(A) for the second polynomial of a double one
            if (op)
                PP_TRY(run_program(A, op, PP_APPLY_PHI, basis, u, w, st));
            else
                PP_TRY(spmv_axpby(A, basis, u, 1.0, nullptr, 0.0, w, st));
        }
        int prow = 0;
        HIP_TRY(launch_dots_pair(basis, n, ws.V, ws.ldv, j, u, last ? u : w, A->partial, A->ldp, A->nblk_dot, &prow,
                                 st));
        HIP_TRY(launch_reduce(prow, A->partial, A->ldp, 2 * j + 2, dd, nullptr, 0, st));
        HIP_TRY(launch_dcgs_step(j, dd, Hdev, ld, pend, coef, last ? 1 : 0, st));
        if (!last)
            HIP_TRY(launch_update_pair(basis, n, ws.V, ws.ldv, j, dd, dd + 2 * j + 2, coef, u, w,
                                       vcol(ws, basis, j), st));
    }
    Hbar.assign((size_t)ld * d, 0.0);
    HIP_TRY(hipMemcpyAsync(Hbar.data(), Hdev, sizeof(double) * ld * d, hipMemcpyDeviceToHost, st));
    HIP_TRY(copy_barrier_flag(A, st));
    HIP_TRY(hipStreamSynchronize(st));
    PP_TRY(check_barrier_flag(A));
    k = d;
    brk = false;
    double fro2 = 0.0;
    dots = 1;
    for (int j = 0; j < d; ++j) {
        dots += 2 * (j + 1) + 2;
        for (int i = 0; i <= j + 1; ++i) {
            const double h = Hbar[(size_t)i + (size_t)j * ld];
            if (!std::isfinite(h)) {
                set_error(std::string(who) + ": non-finite Hessenberg entry");
                return PP_EINVAL;
            }
            fro2 += h * h;
        }
        if (Hbar[(size_t)(j + 1) + (size_t)j * ld] <= kBreakdownTol * std::sqrt(fro2)) {
            k = j + 1;
            brk = true;
            break;
        }
    }
    return PP_OK;
}

// The polynomial of degree kk from the leading (kk+1) x kk block of Hbar
// (Algorithm 4 step 1b, then Algorithm 2): the first kk Arnoldi steps from
// the same start vector are the GMRES(kk) cycle. at_break: the block ends
// at a breakdown (roots are then eig(H_kk)).
pp_status poly_from_hbar(const std::vector<double> &Hbar, int ld, int kk, bool at_break, bool add_roots,
                         const char *who, pp_poly *out) {
    std::vector<double> hk((size_t)(kk + 1) * kk);
    for (int j = 0; j < kk; ++j)
        for (int i = 0; i <= kk; ++i) hk[(size_t)i + (size_t)j * (kk + 1)] = Hbar[(size_t)i + (size_t)j * ld];
    std::vector<double> re(kk), im(kk);
    int hs = harmonic_ritz(kk, hk.data(), at_break, re.data(), im.data());
    if (hs != PP_OK) {
        if (hs == PP_ESINGULAR) set_error(std::string(who) + ": singular H_dd or zero harmonic Ritz value");
        return (pp_status)hs;
    }
    auto *p = new (std::nothrow) pp_poly_s();
    if (!p) return PP_ENOMEM;
    int ps = plan_roots(kk, re.data(), im.data(), add_roots, p->plan);
    if (ps != PP_OK) {
        delete p;
        return (pp_status)ps;
    }
    p->theta_re = re;
    p->theta_im = im;
    p->breakdown = at_break ? 1 : 0;
    p->finalize();
    *out = p;
    return PP_OK;
}

}  // namespace

extern "C" {

pp_status pp_gmres_setup(pp_matrix A, const double *v0, int d, int add_roots, void *stream, pp_poly *out,
                         pp_setup_info *info) {
    if (!A || !v0 || !out || d < 1 || d > A->n || d > kMaxDegree) {
        set_error("pp_gmres_setup: bad argument (need 1 <= d <= min(n, 4096))");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    std::vector<double> Hbar;
    int k = 0;
    bool brk = false;
    int64_t dots = 0;
    PP_TRY(setup_arnoldi(A, v0, d, st, Hbar, k, brk, dots, "pp_gmres_setup"));
    pp_poly p = nullptr;
    PP_TRY(poly_from_hbar(Hbar, d + 1, k, brk, add_roots != 0, "pp_gmres_setup", &p));
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

pp_status pp_gmres_setup_basis(pp_matrix A, const double *v0, int d, int add_roots, int basis, void *stream,
                               pp_poly *out, pp_setup_info *info) {
    if (!A || !v0 || !out || d < 1 || d > A->n || d > kMaxDegree || (basis != PP_F64 && basis != PP_F32)) {
        set_error("pp_gmres_setup_basis: bad argument (need 1 <= d <= min(n, 4096), basis PP_F64 or PP_F32)");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    std::vector<double> Hbar;
    int k = 0;
    bool brk = false;
    int64_t dots = 0;
    PP_TRY(setup_arnoldi(A, v0, d, st, Hbar, k, brk, dots, "pp_gmres_setup_basis", nullptr, basis));
    pp_poly p = nullptr;
    PP_TRY(poly_from_hbar(Hbar, d + 1, k, brk, add_roots != 0, "pp_gmres_setup_basis", &p));
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

pp_status pp_gmres_setup_double(pp_matrix A, pp_poly p1, const double *v0, int d2, int add_roots, void *stream,
                                pp_poly *out, pp_setup_info *info) {
    if (!A || !p1 || !v0 || !out || d2 < 1 || d2 > A->n || d2 > kMaxDegree) {
        set_error("pp_gmres_setup_double: bad argument (need p1 and 1 <= d2 <= min(n, 4096))");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    std::vector<double> Hbar;
    int k = 0;
    bool brk = false;
    int64_t dots = 0;
    PP_TRY(setup_arnoldi(A, v0, d2, st, Hbar, k, brk, dots, "pp_gmres_setup_double", p1));
    pp_poly q = nullptr;
    PP_TRY(poly_from_hbar(Hbar, d2 + 1, k, brk, add_roots != 0, "pp_gmres_setup_double", &q));
    q->inner = std::make_shared<const pp_poly_s>(*p1);
    *out = q;
    if (info) {
        info->d = k;
        info->d_eff = q->plan.d_eff;
        info->n_added = q->plan.n_added;
        info->breakdown = brk ? 1 : 0;
        info->mvps = (int64_t)k * chain_mvps(p1, PP_APPLY_PHI);
        info->dots = dots;
        info->t_setup_s = now_s() - t0;
    }
    return (brk && k < d2) ? PP_BREAKDOWN : PP_OK;
}

pp_status pp_gmres_setup_checked(pp_matrix A, const double *v0, int d, int add_roots, const pp_stch_opts *opts,
                                 void *stream, pp_poly *out, pp_setup_info *info, double *stch) {
    if (!A || !v0 || !out || !opts || !opts->b || d < 1 || d > A->n || d > kMaxDegree || !(opts->tol >= 0.0) ||
        opts->d_step < 0) {
        set_error("pp_gmres_setup_checked: bad argument (need 1 <= d <= min(n, 4096), b, tol >= 0, d_step >= 0)");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    std::vector<double> Hbar;
    int k = 0;
    bool brk = false;
    int64_t dots = 0;
    PP_TRY(setup_arnoldi(A, v0, d, st, Hbar, k, brk, dots, "pp_gmres_setup_checked"));
    double bn = 0.0;
    PP_TRY(dev_norm(A, 0, opts->b, &bn, st));
    const double limit = opts->tol * bn;
    const int d_min = std::max(opts->d_min, 1);
    int64_t mvps = k;
    pp_poly best = nullptr;
    double best_st = 0.0, best_key = 0.0;
    bool stable = false;
    for (int kk = k;;) {
        const bool at_break = brk && kk == k;
        pp_poly p = nullptr;
        pp_status s = poly_from_hbar(Hbar, d + 1, kk, at_break, add_roots != 0, "pp_gmres_setup_checked", &p);
        if (s != PP_OK) {
            if (best) pp_poly_destroy(best);
            return s;
        }
        double sc = 0.0;
        s = pp_stability_check(p, A, opts->b, stream, &sc);
        if (s != PP_OK) {
            pp_poly_destroy(p);
            if (best) pp_poly_destroy(best);
            return s;
        }
        mvps += chain_mvps(p, PP_APPLY_P) + 1 + chain_mvps(p, PP_APPLY_PHI);  // p(A)b, A p(A)b, phi(A)b
        dots += 1;
        const double key = std::isfinite(sc) ? sc : INFINITY;
        if (sc <= limit) {
            if (best) pp_poly_destroy(best);
            best = p;
            best_st = sc;
            stable = true;
            break;
        }
        if (!best || key < best_key) {
            if (best) pp_poly_destroy(best);
            best = p;
            best_st = sc;
            best_key = key;
        } else {
            pp_poly_destroy(p);
        }
        if (opts->d_step <= 0 || kk - opts->d_step < d_min) break;
        kk -= opts->d_step;
    }
    *out = best;
    if (stch) *stch = best_st;
    if (info) {
        info->d = best->plan.d;
        info->d_eff = best->plan.d_eff;
        info->n_added = best->plan.n_added;
        info->breakdown = best->breakdown;
        info->mvps = mvps;
        info->dots = dots;
        info->t_setup_s = now_s() - t0;
    }
    if (!stable) return PP_UNSTABLE;
    return (best->breakdown && k < d) ? PP_BREAKDOWN : PP_OK;
}

pp_status pp_apply(pp_poly p, pp_matrix A, int kind, int prec, const void *v, void *y, void *stream) {
    if (!p || !A || !v || !y || v == y || !valid_prec(prec) || kind < 0 || kind > 2) {
        set_error("pp_apply: bad argument");
        return PP_EINVAL;
    }
    PP_TRY(A->ensure_ws(prec, 0));
    return run_program(A, p, kind, prec, v, y, S(stream));
}

pp_status pp_apply_noalloc(pp_poly p, pp_matrix A, int kind, int prec, const void *v, void *y, void *stream) {
    if (!p || !A || !v || !y || v == y || !valid_prec(prec) || kind < 0 || kind > 2) {
        set_error("pp_apply_noalloc: bad argument");
        return PP_EINVAL;
    }
    if (p->inner) {
        set_error("pp_apply_noalloc: a double polynomial needs more temporaries than the fixed scratch holds");
        return PP_EINVAL;
    }
    if (!A->tuned[prec] || A->persist[prec]) {
        set_error("pp_apply_noalloc: tune (pp_matrix_tune) or set a single-launch variant for this precision first");
        return PP_EINVAL;
    }
    const size_t ldv = ((size_t)A->n + 63) / 64 * 64;
    const size_t vec = ldv * elem_size(prec);
    if (3 * vec > kNoallocScratchBytes) {
        set_error("pp_apply_noalloc: 3 temporaries of " + std::to_string(vec) + " bytes exceed the " +
                  std::to_string(kNoallocScratchBytes) + "-byte scratch (n <= " +
                  std::to_string(kNoallocScratchBytes / 3 / elem_size(prec) / 64 * 64) + " in this precision)");
        return PP_EINVAL;
    }
    char *base = nullptr;
    PP_TRY(noalloc_scratch(&base));
    void *const temps[3] = {base, base + vec, base + 2 * vec};
    return run_program(A, p, kind, prec, v, y, S(stream), temps);
}

pp_status pp_chain_bytes(pp_poly p, pp_matrix A, int kind, int prec, void *stream, int64_t *bytes,
                         int64_t *launches) {
    if (!p || !A || !bytes || !valid_prec(prec) || kind < 0 || kind > 2) {
        set_error("pp_chain_bytes: bad argument");
        return PP_EINVAL;
    }
    PP_TRY(ensure_tuned(A, prec, S(stream)));
    int64_t b = 0, l = 0;
    program_bytes(A, p, kind, prec, b, l);
    *bytes = b;
    if (launches) *launches = l;
    return PP_OK;
}

pp_status pp_solve_workspace_bytes(pp_poly p, pp_matrix A, const pp_solve_opts *opts, int64_t *total,
                                   int64_t *additional) {
    const int d_new = opts ? opts->new_poly_degree : 0;
    if (!A || !opts || opts->m < 1 || !valid_prec(opts->inner) || d_new < 0 || d_new > std::min(A->n, kMaxDegree) ||
        (!p && d_new <= 0)) {
        set_error("pp_solve_workspace_bytes: bad argument");
        return PP_EINVAL;
    }
    const int64_t ldv = ((int64_t)A->n + 63) / 64 * 64;
    int64_t tot = 0, add = 0;
    // Krylov basis (m + 1 columns) and 5 work vectors per precision a cycle
    // may run in (FP64 always: refinement falls back to it; ChPoly's setup
    // needs d_new + 1 columns of it), plus 5 more for a composite polynomial
    auto ws = [&](int prec, int cols) {
        const int64_t b = ldv * (int64_t)elem_size(prec) * (cols + 1 + 5);
        const int64_t x = (p && p->inner) ? ldv * (int64_t)elem_size(prec) * 5 : 0;
        tot += b + x;
        const Workspace &w = A->ws[prec];
        if (!(w.m >= cols && w.P0)) add += b + (w.X ? 0 : x);
        else if (x && !w.X) add += x;
    };
    ws(0, std::max(opts->m, d_new));
    if (opts->inner != PP_F64) ws(opts->inner, opts->m);
    // reduction buffers (device) for the widest Gram-Schmidt pass
    const int cols = std::max(std::max(opts->m, d_new) + 1, d_new > 0 ? 2 * d_new + 4 : 0);
    const int64_t want = std::max(cols + 2, 64);
    const int64_t red = (int64_t)sizeof(double) * want * (std::max(A->nblk_dot, A->nblk_ud) + 5);
    tot += red;
    if (cols + 2 > A->ldp) add += red;
    // ChPoly: each cycle's setup holds its (d+1) x d Hessenberg matrix
    if (d_new > 0) {
        const int64_t h = (int64_t)sizeof(double) * (d_new + 1) * d_new;
        tot += h;
        add += h;
    }
    if (total) *total = tot;
    if (additional) *additional = add;
    return PP_OK;
}

pp_status pp_launch_floor(int launches, int64_t blocks, int threads, void *stream) {
    if (launches < 1 || launches > 100000 || blocks < 1 || blocks >= (1LL << 31) ||
        (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)) {
        set_error("pp_launch_floor: bad argument");
        return PP_EINVAL;
    }
    for (int i = 0; i < launches; ++i) HIP_TRY(launch_empty((long)blocks, threads, S(stream)));
    return PP_OK;
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
    PP_TRY(run_program(A, p, PP_APPLY_P, 0, b, ws.D, st));
    PP_TRY(spmv_axpby(A, 0, ws.D, -1.0, b, 1.0, ws.ACC, st));
    PP_TRY(run_program(A, p, PP_APPLY_PI, 0, b, A->r64, st));
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
    const int d_new = opts ? opts->new_poly_degree : 0;
    if ((!p && d_new <= 0) || !A || !b || !x || !opts || opts->m < 1 || opts->max_cycles < 0 ||
        !(opts->tol > 0.0) || !valid_prec(opts->inner) || d_new < 0 || d_new > std::min(A->n, kMaxDegree)) {
        set_error("pp_solve: bad argument");
        return PP_EINVAL;
    }
    hipStream_t st = S(stream);
    const double t0 = now_s();
    const int n = A->n;
    const int m = opts->m;
    PP_TRY(A->ensure_ws(0, std::max(m, d_new)));
    if (opts->inner != PP_F64) PP_TRY(A->ensure_ws(opts->inner, m));
    PP_TRY(A->ensure_red(std::max(m, d_new) + 1));
    // ChPoly: the polynomial of the current cycle, owned here
    struct Owned {
        pp_poly q = nullptr;
        ~Owned() {
            if (q) pp_poly_destroy(q);
        }
    } owned;
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
    // marks the arrival of a Hessenberg column in host memory
    struct Ev {
        hipEvent_t e = nullptr;
        ~Ev() {
            if (e) (void)hipEventDestroy(e);
        }
    } col_ready;
    HIP_TRY(hipEventCreateWithFlags(&col_ready.e, hipEventDisableTiming));
    int prec = opts->inner;
    std::vector<double> hist;
    GivensLS ls;
    std::vector<double> zh(m + 1);
    pp_status status = PP_OK;
    for (;;) {
        const double relres = beta / bnorm;
        if (opts->history && (int)hist.size() < opts->history_cap) opts->history[hist.size()] = relres;
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
        if (d_new > 0) {
            // section 5.2: a new polynomial from GMRES(d) started at the current residual
            std::vector<double> Hb;
            int kk = 0;
            bool brk = false;
            int64_t sdots = 0;
            PP_TRY(setup_arnoldi(A, A->r64, d_new, st, Hb, kk, brk, sdots, "pp_solve"));
            pp_poly q = nullptr;
            PP_TRY(poly_from_hbar(Hb, d_new + 1, kk, brk, opts->new_poly_add != 0, "pp_solve", &q));
            if (owned.q) pp_poly_destroy(owned.q);
            owned.q = q;
            p = q;
            inf.mvps += kk;
            inf.dots += sdots;
        }
        const int64_t mv_phi = chain_mvps(p, PP_APPLY_PHI), mv_p = chain_mvps(p, PP_APPLY_P);
        const Workspace &ws = A->ws[prec];
        // V[:,0] = r / beta in the cycle's precision
        HIP_TRY(launch_scale_cast(0, prec, n, A->r64, nullptr, 1.0 / beta, vcol(ws, prec, 0), st));
        ls.reset(m, beta);
        const double eta = (prec != PP_F64 && opts->inner_eta > 0.0) ? opts->inner_eta : kInnerEta[prec];
        const double target = std::max(opts->tol * bnorm, eta * beta);
        double fro2 = 0.0;
        int k = 0;
        // lookahead: phi(A) V[:, j] already queued; the last shortcut
        // residual and the last step's reduction factor. A wrong guess costs
        // a whole phi(A) application, a right one saves a host round trip:
        // queue ahead only while the predicted residual is above the target
        // by more than that ratio.
        bool ahead = false;
        double r_last = beta, rate = 1.0;
        const double t_phi = (double)chain_launches(p, PP_APPLY_PHI) *
                             (A->tuned_us[prec] > 0.0 ? A->tuned_us[prec] : kLaunchGuessUs);
        const double margin = std::max(2.0, t_phi / kLookaheadGapUs);
        for (int j = 0; j < m; ++j) {
            if (!ahead) PP_TRY(run_program(A, p, PP_APPLY_PHI, prec, vcol(ws, prec, j), vcol(ws, prec, j + 1), st));
            PP_TRY(cgs2_step(A, prec, ws, j, st, nullptr, false));
            HIP_TRY(hipMemcpyAsync(A->hpin, A->H(), sizeof(double) * (j + 2), hipMemcpyDeviceToHost, st));
            HIP_TRY(copy_barrier_flag(A, st));
            HIP_TRY(hipEventRecord(col_ready.e, st));
            // V[:, j+1] is final once the step's kernels ran: queue the next
            // step's product unless this step is expected to end the cycle
            // (not on a cycle's first step: no reduction factor is known yet,
            // and a strong polynomial may end the cycle there)
            ahead = opts->lookahead && j >= 1 && j + 1 < m && r_last * rate > margin * target;
            if (ahead)
                PP_TRY(run_program(A, p, PP_APPLY_PHI, prec, vcol(ws, prec, j + 1), vcol(ws, prec, j + 2), st));
            HIP_TRY(hipEventSynchronize(col_ready.e));
            PP_TRY(check_barrier_flag(A));
            inf.mvps += mv_phi;
            inf.dots += 2 * (j + 1) + 1;
            inf.vops += 4 * (j + 1) + 2 + chain_launches(p, PP_APPLY_PHI);
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
            rate = r_last > 0.0 ? shortcut / r_last : 1.0;
            r_last = shortcut;
            const bool lucky = A->hpin[j + 1] <= kBreakdownTol * std::sqrt(fro2);
            if (lucky || shortcut <= target) break;
        }
        if (ahead) inf.lookahead_discarded++;  // a queued product the cycle did not need
        if (k > 0) {
            ls.solve(zh.data());
            // stage through pinned memory: the host reads the staging slot
            // below only after the stream passed the column's copy; a queued
            // product may still run, and the upload is ordered after it
            std::memcpy(A->hpin + A->ldp, zh.data(), sizeof(double) * k);
            HIP_TRY(hipMemcpyAsync(A->z(), A->hpin + A->ldp, sizeof(double) * k, hipMemcpyHostToDevice, st));
            // dy = V_k z (z solves min ||beta e1 - Hbar z||, so it carries beta);
            // dx = p(A) dy ; x += dx in FP64
            HIP_TRY(launch_combine(prec, n, ws.V, ws.ldv, k, A->z(), ws.D, st));
            PP_TRY(run_program(A, p, PP_APPLY_P, prec, ws.D, ws.ACC, st));
            HIP_TRY(launch_axpy_x(prec, n, 1.0, ws.ACC, x, st));
            inf.mvps += mv_p;
            inf.vops += k + chain_launches(p, PP_APPLY_P) * 2 + 1;
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
    // composition with a right preconditioner: x = diag(s) x~ (eq. (1.4))
    if (A->scale_mode != 0) HIP_TRY(launch_vmul(n, x, A->scale, st));
    // composition with block-Jacobi: x = M^{-1} x~
    if (A->rbs > 0) HIP_TRY(launch_block_apply(n, A->rbs, A->rminv, x, st));
    inf.status = status;
    inf.t_solve_s = now_s() - t0;
    if (info) *info = inf;
    return status;
}

}  // extern "C"
