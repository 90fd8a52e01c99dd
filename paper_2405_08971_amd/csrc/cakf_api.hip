// C ABI of libcakf: context management and the orchestration of one filter step
// (Alg. 1: predict, update, truncate) on one HIP stream.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <mutex>
#include <new>

#include "../../include/cakf.h"
#include "cakf_common.h"
#include "launchers.h"

using namespace cakf;

namespace {

inline int round_up(int v, int a) { return (v + a - 1) / a * a; }

struct Diag {
    int dropped;
    int nonfinite;
    int bad_index;
    int steps;          // updates with data since the last reset
    double loglik;      // sum of the projected log-likelihood terms since the last reset
};

// Per-phase timing with HIP events recorded on the context stream around each launch.
struct Prof {
    static constexpr int CAP = 2048;
    hipEvent_t* ev[CAKF_PHASES][2];
    int count[CAKF_PHASES];
    int mask;           // bit p: phase p is timed
    int stride;         // time every stride-th launch of a timed phase (>= 1)
    int seen[CAKF_PHASES];
    bool on;
};

}  // namespace

struct cakf_ctx {
    cakf_config cfg;
    hipStream_t stream;
    rocblas_handle blas;
    int device;
    // dimensions
    int n, r, imax, mmax, mpmax, ldM, bp, Kmax, ldmo, gs;
    size_t gram_work_elems;
    // state
    float* mean;
    float* M[2];
    int cur;          // index of the buffer holding the factor
    int rank;
    // the first orth columns of the factor are mutually orthogonal with squared norms
    // orth_scale * lam[c]: the columns M V_r of the last truncation, scaled by the
    // predictions since (0 when not known)
    int orth;
    double orth_scale;
    double* lam;
    // observation space workspace
    float4* Xs;
    float4* Xo;
    float* r0;
    float* Mo;
    float* S;
    float* U;
    float* V;
    float* T;
    float* part;
    double* cpart;     // next_action's per-block column products
    double* colvec;    // the reduced column products of the current action
    double* fupart;    // per-row-block sums of s_j^T u_j (action-loop step)
    double* tri;       // triangular products of the current action's Cholesky step
    unsigned* ctr;     // arrival counter of the sym_tiles spare blocks (zero between launches)
    double* ttpart;    // the spare blocks' shares of T^T t_j
    double* beta2;     // beta after odd actions (c->beta: after even actions, and final)
    double* SS;        // S^T S of the current update's actions (rows l <= j)
    double* SSwork;    // its factorisation once the loop ends, when too large for LDS
    float* mpart;
    double *Linv, *LinvT, *L, *LSinv, *LSinvT, *alpha, *beta;
    LoopState* ls;
    Diag* diag;
    // block product
    float* B;
    float* Q;
    __bf16* Bth;
    __bf16* Btl;
    // truncation
    double* G;
    double* gwork;
    double* eigval;
    double* offdiag;
    int* info;
    float* Vr;
    // tridiagonalisation (K <= TD_MAXK): reflectors, tau, exchange vectors, barrier words
    double *tdV, *tdtau, *tdp, *tdrow;
    unsigned* tdctr;
    int* tdabort;
    void* blas_ws;
    Prof prof;
    // smoother (allocated when cfg.smoother != 0)
    int np, bps, ldWs;
    float4* Xp;
    float* sm_ws;
    float* sm_W[2];
    int sm_cur, sm_rank;
    bool sm_started;
    float *sm_B, *sm_Y, *sm_Z, *sm_Q, *sm_Gr, *sm_R, *sm_WR;
    __bf16 *sm_Bth, *sm_Btl;
    // log-likelihood derivative (allocated when cfg.gradient != 0)
    float* gMb[2];     // adjoint of the factor (n x ldM), ping-pong
    float* gmb;        // adjoint of the mean (n)
    float* gYb;        // adjoint of the new columns and the mean increment (n x bp)
    float *gBq, *gBb;  // B = [W w] and its adjoint (mpmax x bp)
    float* gbpart;     // per-slice partials of K(Xo, X) Ybar
    size_t gbpart_elems;
    double* gspart;    // per-block partial sums of the tile kernels
    int gspart_blocks;
    float *gQb, *gMob, *gZr, *gCc;
    double *gW64, *gSr64, *gBb64, *gG1, *gG2, *gX1, *gX2, *gpart, *gacc;
    double* gatb;      // slab partials of the FP64 products G1, G2
    // path sampler (allocated when cfg.sample_paths > 0)
    int sp_ns, bsp;
    float *sp_B, *sp_W, *sp_Y, *sp_D, *sp_D2, *sp_R, *sp_Z, *sp_Q;
    __bf16 *sp_Bth, *sp_Btl;
    float4* sp_Xo;
    int N;            // state rows: n, or 2n with the Matérn-3/2 temporal factor
    // partial products of block products split along the observation axis
    float* bpart;
    size_t bpart_elems;
    // block-residual policy (allocated when cfg.policy == CAKF_POLICY_BLOCK)
    int bmax, ldz;
    double* bpart64;  // slab partials of the round's Gram product
    float* bpart32;   // slab partials of Mo^T S_round
    double* bG;       // S^T [U_r | S_r | V_r | r0] of the round (imax x ldz)
};

namespace {

// Whether this launch of phase ph is timed (the phase is enabled, this launch falls on
// the sampling stride and an event pair is free).
bool prof_take(cakf_ctx* c, int ph) {
    if (!c->prof.on || !(c->prof.mask >> ph & 1)) return false;
    const bool on_stride = c->prof.seen[ph]++ % c->prof.stride == 0;
    return on_stride && c->prof.count[ph] < Prof::CAP;
}

struct PhaseTimer {
    cakf_ctx* c;
    int ph;
    bool take;
    PhaseTimer(cakf_ctx* c_, int ph_) : c(c_), ph(ph_), take(prof_take(c_, ph_)) {
        if (take) (void)hipEventRecord(c->prof.ev[ph][0][c->prof.count[ph]], c->stream);
    }
    ~PhaseTimer() {
        if (take) {
            (void)hipEventRecord(c->prof.ev[ph][1][c->prof.count[ph]], c->stream);
            ++c->prof.count[ph];
        }
    }
};

// Timing of a phase that is one kernel launch: hands out the event pair, which the launch
// stamps with its own start and stop times (hipExtLaunchKernel), so the figure is the
// kernel's duration without the event packets around it.
struct KernelTimer {
    cakf_ctx* c;
    int ph;
    hipEvent_t start = nullptr, stop = nullptr;
    KernelTimer(cakf_ctx* c_, int ph_) : c(c_), ph(ph_) {
        if (prof_take(c, ph)) {
            start = c->prof.ev[ph][0][c->prof.count[ph]];
            stop = c->prof.ev[ph][1][c->prof.count[ph]];
        }
    }
    ~KernelTimer() {
        if (start) ++c->prof.count[ph];
    }
};

void prof_free(cakf_ctx* c) {
    for (int p = 0; p < CAKF_PHASES; ++p)
        for (int k = 0; k < 2; ++k)
            if (c->prof.ev[p][k]) {
                for (int e = 0; e < Prof::CAP; ++e) (void)hipEventDestroy(c->prof.ev[p][k][e]);
                delete[] c->prof.ev[p][k];
                c->prof.ev[p][k] = nullptr;
            }
    c->prof.on = false;
}

}  // namespace

#define HIP_TRY(x)                                   \
    do {                                             \
        if ((x) != hipSuccess) return CAKF_E_HIP;    \
    } while (0)
#define BLAS_TRY(x)                                          \
    do {                                                     \
        if ((x) != rocblas_status_success) return CAKF_E_SOLVER; \
    } while (0)

static void free_all(cakf_ctx* c) {
    void* ptrs[] = {c->mean, c->M[0], c->M[1], c->Xs, c->Xo, c->r0, c->Mo, c->S, c->U, c->V, c->T,
                    c->part, c->cpart, c->colvec, c->fupart, c->tri, c->ctr, c->ttpart, c->beta2, c->SS, c->SSwork, c->mpart, c->Linv,
                    c->LinvT, c->L, c->LSinv, c->LSinvT,
                    c->alpha, c->beta, c->ls, c->diag, c->B, c->Q, c->Bth, c->Btl, c->G, c->gwork, c->eigval,
                    c->lam, c->offdiag, c->info, c->Vr, c->tdV, c->tdtau, c->tdp, c->tdrow, c->tdctr,
                    c->tdabort, c->blas_ws, c->Xp, c->sm_ws, c->sm_W[0],
                    c->sm_W[1], c->sm_B, c->sm_Y, c->sm_Z, c->sm_Q, c->sm_Gr, c->sm_R,
                    c->sm_WR, c->sm_Bth, c->sm_Btl, c->gMb[0], c->gMb[1], c->gmb, c->gYb,
                    c->gBq, c->gBb, c->gbpart, c->gspart, c->gQb, c->gMob, c->gZr, c->gCc,
                    c->gW64, c->gSr64, c->gBb64, c->gG1, c->gG2, c->gX1, c->gX2, c->gpart,
                    c->gacc, c->gatb, c->bpart64, c->bpart32, c->bG, c->bpart, c->sp_B,
                    c->sp_W, c->sp_Y, c->sp_D, c->sp_D2, c->sp_R, c->sp_Z, c->sp_Q, c->sp_Bth,
                    c->sp_Btl, c->sp_Xo};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

template <typename Tp>
static int dalloc(Tp** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(Tp)) != hipSuccess) {
        *p = nullptr;
        return CAKF_E_NOMEM;
    }
    return CAKF_OK;
}

static int validate(const cakf_config* c) {
    if (!c || !c->X) return CAKF_E_ARG;
    if (c->n < 1 || (c->dim != 2 && c->dim != 3)) return CAKF_E_ARG;
    if (c->kernel != CAKF_MATERN12 && c->kernel != CAKF_MATERN32 && c->kernel != CAKF_MATERN52)
        return CAKF_E_ARG;
    if (c->dist != CAKF_DIST_EUCLID && c->dist != CAKF_DIST_GEODESIC) return CAKF_E_ARG;
    if (c->dist == CAKF_DIST_GEODESIC && c->dim != 3) return CAKF_E_ARG;
    if (!(c->lengthscale > 0) || !(c->signal_var > 0) || !(c->noise_var > 0)) return CAKF_E_ARG;
    if (!(c->ou_coeff > 0) || c->ou_coeff > 1) return CAKF_E_ARG;
    if (c->max_obs < 1 || c->max_actions < 1 || c->max_actions > 256) return CAKF_E_ARG;
    if (c->max_rank < 1 || c->max_rank > 1024) return CAKF_E_ARG;
    if (c->policy != CAKF_POLICY_CG && c->policy != CAKF_POLICY_GIVEN &&
        c->policy != CAKF_POLICY_BLOCK)
        return CAKF_E_ARG;
    if (c->policy == CAKF_POLICY_BLOCK &&
        (c->block_actions < 1 || c->block_actions > c->max_actions))
        return CAKF_E_ARG;
    // the residual-tolerance stop reads ||r_j||^2 = s_j^T s_j, which holds only when the
    // actions are the residuals (CG)
    if (c->resid_tol != 0 && c->policy != CAKF_POLICY_CG) return CAKF_E_ARG;
    if (c->prec != CAKF_PREC_FP32 && c->prec != CAKF_PREC_BF16 && c->prec != CAKF_PREC_BF16X3)
        return CAKF_E_ARG;
    if (c->resid_tol < 0 || c->pivot_tol < 0) return CAKF_E_ARG;
    if (c->smoother && (size_t)c->n * (c->max_rank + 1) > ((size_t)1 << 31)) return CAKF_E_ARG;
    // the reverse sweep's FP64 Cholesky adjoint keeps per-action vectors of 256 in LDS
    if (c->gradient && c->max_actions > 256) return CAKF_E_ARG;
    if (c->sample_paths < 0 || c->sample_paths > 256) return CAKF_E_ARG;
    if (c->temporal != CAKF_TEMPORAL_OU && c->temporal != CAKF_TEMPORAL_MATERN32)
        return CAKF_E_ARG;
    if (c->temporal == CAKF_TEMPORAL_MATERN32 &&
        (c->smoother || c->gradient || c->sample_paths > 0))
        return CAKF_E_ARG;
    return CAKF_OK;
}

// ------------------------------------------------------- static scratch (no allocation)
// The workspace of cakf_sample_forward_static: a file-scope device array of
// CAKF_STATIC_SCRATCH_BYTES, one copy per GPU, held until the process ends.  In host code
// the array's name is not a device address: the address of the current device's copy is
// looked up once per device (cakf_create, with that device current) and only that address
// is handed to kernels and library calls.
static __device__ __align__(256) unsigned char scratch[CAKF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_addr[SCRATCH_MAX_DEVICES];
bool scratch_looked_up[SCRATCH_MAX_DEVICES];

// Device address of this device's scratch copy (dev must be the current device).
void scratch_lookup(int dev) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return;
    std::lock_guard<std::mutex> guard(scratch_mu);
    if (scratch_looked_up[dev]) return;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) {
        scratch_addr[dev] = p;
        scratch_looked_up[dev] = true;
    } else {
        (void)hipGetLastError();   // leave no error behind for later calls
    }
}

void* scratch_of(int dev) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> guard(scratch_mu);
    return scratch_addr[dev];
}

// Bump allocation of 256-byte aligned segments inside [base, base + cap).
struct Carve {
    char* base;
    size_t cap, used = 0;
    bool ok = true;
    template <typename Tp>
    Tp* take(size_t count) {
        const size_t bytes = (count * sizeof(Tp) + 255) / 256 * 256;
        if (!ok || bytes > cap - used) {
            ok = false;
            return nullptr;
        }
        Tp* p = reinterpret_cast<Tp*>(base + used);
        used += bytes;
        return p;
    }
};
}  // namespace

extern "C" int cakf_create(const cakf_config* cfg, cakf_ctx** out) {
    if (!out) return CAKF_E_ARG;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    cakf_ctx* c = new (std::nothrow) cakf_ctx;
    if (!c) return CAKF_E_NOMEM;
    std::memset(c, 0, sizeof(*c));
    c->prof.stride = 1;
    c->cfg = *cfg;
    c->stream = (hipStream_t)cfg->stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return CAKF_E_HIP;
    }
    // the static scratch array's address on this device (cakf_sample_forward_static)
    scratch_lookup(c->device);
    c->n = cfg->n;
    c->N = cfg->temporal == CAKF_TEMPORAL_MATERN32 ? 2 * cfg->n : cfg->n;
    c->r = cfg->max_rank;
    c->imax = cfg->max_actions;
    c->mmax = cfg->max_obs;
    c->mpmax = round_up(c->mmax, SYM_TILE);
    c->ldM = round_up(c->r + c->imax + 1, 4);
    c->bp = round_up(c->imax + 1, 32);
    c->Kmax = c->r + c->imax;
    c->ldmo = round_up(c->r, 8);
    c->gs = 2 * c->imax + 2;
    c->gram_work_elems = (size_t)16 * c->Kmax * c->Kmax;
    const size_t n = c->n;
    const int nbmax = c->mpmax / SYM_TILE;
    // largest block count of a next_action launch (the column-product and Mo^T s partials)
    const int nablk = std::max(next_action_blocks(c->mmax, 4, 4), next_action_blocks(c->mmax, 16, 1));
    rc = CAKF_OK;
    rc |= dalloc(&c->mean, (size_t)c->N);
    rc |= dalloc(&c->M[0], (size_t)c->N * c->ldM);
    rc |= dalloc(&c->M[1], (size_t)c->N * c->ldM);
    rc |= dalloc(&c->Xs, n);
    rc |= dalloc(&c->Xo, c->mpmax);
    rc |= dalloc(&c->r0, c->mpmax);
    rc |= dalloc(&c->Mo, (size_t)c->mpmax * c->ldmo);
    rc |= dalloc(&c->S, (size_t)c->mpmax * c->imax);
    rc |= dalloc(&c->U, (size_t)c->mpmax * c->imax);
    rc |= dalloc(&c->V, (size_t)c->mpmax * c->imax);
    rc |= dalloc(&c->T, (size_t)c->ldmo * c->imax);
    rc |= dalloc(&c->part, (size_t)nbmax * c->mpmax);
    rc |= dalloc(&c->cpart, (size_t)nablk * c->gs);
    rc |= dalloc(&c->colvec, (size_t)c->gs);
    rc |= dalloc(&c->fupart, (size_t)nbmax);
    rc |= dalloc(&c->tri, (size_t)tri_elems(c->imax));
    rc |= dalloc(&c->ctr, 1);
    rc |= dalloc(&c->ttpart, (size_t)((c->ldmo + 31) / 32) * c->imax);
    rc |= dalloc(&c->beta2, c->imax);
    rc |= dalloc(&c->SS, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->SSwork, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->mpart, (size_t)std::max(nablk, (c->mmax + 63) / 64) * c->ldmo);
    rc |= dalloc(&c->Linv, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->LinvT, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->L, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->LSinv, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->LSinvT, (size_t)c->imax * c->imax);
    rc |= dalloc(&c->alpha, c->imax);
    rc |= dalloc(&c->beta, c->imax);
    rc |= dalloc(&c->ls, 1);
    rc |= dalloc(&c->diag, 1);
    rc |= dalloc(&c->B, (size_t)c->mpmax * c->bp);
    rc |= dalloc(&c->Q, (size_t)c->r * c->bp);
    rc |= dalloc(&c->Bth, (size_t)c->mpmax * c->bp);
    rc |= dalloc(&c->Btl, (size_t)c->mpmax * c->bp);
    rc |= dalloc(&c->G, (size_t)c->Kmax * c->Kmax);
    rc |= dalloc(&c->gwork, c->gram_work_elems);
    rc |= dalloc(&c->eigval, c->Kmax);
    rc |= dalloc(&c->lam, std::max(c->r, 1));
    rc |= dalloc(&c->offdiag, c->Kmax);
    rc |= dalloc(&c->info, 1);
    rc |= dalloc(&c->Vr, (size_t)c->Kmax * c->r);
    if (c->Kmax >= 3 && c->Kmax <= TD_MAXK) {
        rc |= dalloc(&c->tdV, (size_t)c->Kmax * c->Kmax);
        rc |= dalloc(&c->tdtau, c->Kmax);
        rc |= dalloc(&c->tdp, 2 * (size_t)c->Kmax);
        rc |= dalloc(&c->tdrow, 2 * (size_t)c->Kmax);
        rc |= dalloc(&c->tdctr, 1);
        rc |= dalloc(&c->tdabort, 1);
    }
    if (cfg->smoother || cfg->sample_paths > 0) {
        c->np = round_up(c->n, SYM_TILE);
        rc |= dalloc(&c->Xp, c->np);
    }
    if (cfg->sample_paths > 0) {
        c->sp_ns = cfg->sample_paths;
        c->bsp = round_up(cfg->sample_paths, 32);
        const size_t rows = std::max<size_t>(c->np, c->mpmax);
        rc |= dalloc(&c->sp_B, (size_t)c->mpmax * c->bsp);
        rc |= dalloc(&c->sp_W, (size_t)c->np * c->bsp);
        rc |= dalloc(&c->sp_Y, n * c->bsp);
        rc |= dalloc(&c->sp_D, (size_t)c->mpmax * c->bsp);
        rc |= dalloc(&c->sp_D2, (size_t)c->mpmax * c->bsp);
        rc |= dalloc(&c->sp_R, (size_t)c->imax * c->bsp);
        rc |= dalloc(&c->sp_Z, (size_t)c->imax * c->bsp);
        rc |= dalloc(&c->sp_Q, (size_t)c->Kmax * c->bsp);
        rc |= dalloc(&c->sp_Bth, rows * c->bsp);
        rc |= dalloc(&c->sp_Btl, rows * c->bsp);
        rc |= dalloc(&c->sp_Xo, c->mpmax);
    }
    if (cfg->smoother) {
        c->bps = round_up(1 + c->r, 32);
        c->ldWs = round_up(c->imax + c->r, 4);
        rc |= dalloc(&c->sm_ws, n);
        rc |= dalloc(&c->sm_W[0], n * c->ldWs);
        rc |= dalloc(&c->sm_W[1], n * c->ldWs);
        rc |= dalloc(&c->sm_B, (size_t)c->np * c->bps);
        rc |= dalloc(&c->sm_Y, n * c->bps);
        rc |= dalloc(&c->sm_Z, n * c->bps);
        rc |= dalloc(&c->sm_Q, (size_t)c->Kmax * c->bps);
        rc |= dalloc(&c->sm_Gr, (size_t)c->mmax * c->bps);
        rc |= dalloc(&c->sm_R, (size_t)c->imax * c->bps);
        rc |= dalloc(&c->sm_WR, (size_t)c->mmax * c->bps);
        rc |= dalloc(&c->sm_Bth, (size_t)c->np * c->bps);
        rc |= dalloc(&c->sm_Btl, (size_t)c->np * c->bps);
    }
    if (cfg->gradient) {
        const size_t I = c->imax, I1 = c->imax + 1;
        rc |= dalloc(&c->gMb[0], n * c->ldM);
        rc |= dalloc(&c->gMb[1], n * c->ldM);
        rc |= dalloc(&c->gmb, n);
        rc |= dalloc(&c->gYb, n * c->bp);
        rc |= dalloc(&c->gBq, (size_t)c->mpmax * c->bp);
        rc |= dalloc(&c->gBb, (size_t)c->mpmax * c->bp);
        // slices x (m rounded to 32) <= 2048 x 32 + mpmax rows of partials
        c->gbpart_elems = ((size_t)2048 * 32 + c->mpmax) * c->bp;
        rc |= dalloc(&c->gbpart, c->gbpart_elems);
        c->gspart_blocks = adj_tiles_launches(I1) * (2048 + c->mpmax / 32 + 1);
        rc |= dalloc(&c->gspart, (size_t)2 * c->gspart_blocks);
        rc |= dalloc(&c->gQb, (size_t)c->r * c->bp);
        rc |= dalloc(&c->gMob, (size_t)c->mpmax * c->ldmo);
        rc |= dalloc(&c->gZr, (size_t)c->mpmax * I1);
        rc |= dalloc(&c->gCc, I * I1);
        rc |= dalloc(&c->gW64, (size_t)c->mpmax * I);
        rc |= dalloc(&c->gSr64, (size_t)c->mpmax * I1);
        rc |= dalloc(&c->gBb64, (size_t)c->mpmax * I1);
        rc |= dalloc(&c->gG1, I * I1);
        rc |= dalloc(&c->gG2, I * I1);
        rc |= dalloc(&c->gX1, I * I);
        rc |= dalloc(&c->gX2, I * I);
        rc |= dalloc(&c->gpart, (n + 3) / 4);
        rc |= dalloc(&c->gacc, 4);
        rc |= dalloc(&c->gatb, atb64_part_elems(c->mmax, I, I1));
    }
    {
        // Block products with few row blocks are split along the observation axis (see
        // launch_block_product); size their partial buffer for the largest split, capped.
        const size_t unlimited = ~(size_t)0, cap = (size_t)32 << 20;
        auto need_of = [&](int rows, int mp, int cols) -> size_t {
            const int ns = block_product_splits(rows, mp, cols, unlimited);
            return ns > 1 ? (size_t)ns * rows * cols : 0;
        };
        size_t need = need_of(c->n, c->mpmax, c->bp);
        if (cfg->policy == CAKF_POLICY_BLOCK)
            need = std::max(need, need_of(c->mpmax, c->mpmax, cfg->block_actions));
        if (cfg->smoother)
            need = std::max(need, need_of(c->n, round_up(c->n, SYM_TILE), round_up(1 + c->r, 32)));
        if (cfg->sample_paths > 0) {
            const int bsp = round_up(cfg->sample_paths, 32);
            need = std::max(need, need_of(c->n, round_up(c->n, SYM_TILE), bsp));
            need = std::max(need, need_of(c->n, c->mpmax, bsp));
        }
        c->bpart_elems = std::min(need, cap);
        if (c->bpart_elems) rc |= dalloc(&c->bpart, c->bpart_elems);
    }
    if (cfg->policy == CAKF_POLICY_BLOCK) {
        c->bmax = cfg->block_actions;
        c->ldz = 3 * c->bmax + 1;
        rc |= dalloc(&c->bpart64, round_products_elems(c->mmax, c->imax, c->ldz));
        rc |= dalloc(&c->bpart32, round_products_elems(c->mmax, c->r, c->bmax));
        rc |= dalloc(&c->bG, (size_t)c->imax * c->ldz);
    }
    if (rc) {
        free_all(c);
        delete c;
        return CAKF_E_NOMEM;
    }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        free_all(c);
        delete c;
        return CAKF_E_SOLVER;
    }
    rocblas_set_stream(c->blas, c->stream);
    rocblas_set_atomics_mode(c->blas, rocblas_atomics_not_allowed);
    rocblas_set_pointer_mode(c->blas, rocblas_pointer_mode_host);
    // Size the library workspace once (largest eigenproblem) so no later call allocates.
    size_t ws = 0;
    rocblas_start_device_memory_size_query(c->blas);
    rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_lower, c->Kmax, c->G,
                     c->Kmax, c->eigval, c->offdiag, c->info);
    rocsolver_dstedc(c->blas, rocblas_evect_tridiagonal, c->Kmax, c->eigval, c->offdiag, c->G,
                     c->Kmax, c->info);
    rocsolver_dormtr(c->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                     c->Kmax, c->r, c->G, c->Kmax, c->eigval, c->G, c->Kmax);
    rocblas_stop_device_memory_size_query(c->blas, &ws);
    ws = std::max<size_t>(ws, 1 << 20);
    if (hipMalloc(&c->blas_ws, ws) != hipSuccess ||
        rocblas_set_workspace(c->blas, c->blas_ws, ws) != rocblas_status_success) {
        rocblas_destroy_handle(c->blas);
        free_all(c);
        delete c;
        return CAKF_E_NOMEM;
    }
    // Pre-scaled points and the prior state.
    const int nu2 = cfg->kernel;
    const double scale = 1.4426950408889634 * std::sqrt((double)nu2) / cfg->lengthscale;
    launch_prescale(cfg->X, c->n, cfg->dim, (float)scale, cfg->dist, c->Xs, c->stream);
    if (c->Xp) launch_pad_points(c->Xs, c->n, c->np, c->Xp, c->stream);
    if (hipMemsetAsync(c->mean, 0, (size_t)c->N * sizeof(float), c->stream) != hipSuccess ||
        hipMemsetAsync(c->diag, 0, sizeof(Diag), c->stream) != hipSuccess ||
        hipMemsetAsync(c->ctr, 0, sizeof(unsigned), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        rocblas_destroy_handle(c->blas);
        free_all(c);
        delete c;
        return CAKF_E_HIP;
    }
    c->cur = 0;
    c->rank = 0;
    c->orth = 0;
    c->orth_scale = 1.0;
    *out = c;
    return CAKF_OK;
}

extern "C" void cakf_destroy(cakf_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    prof_free(c);
    rocblas_destroy_handle(c->blas);
    free_all(c);
    delete c;
}

extern "C" int cakf_reset(cakf_ctx* c) {
    if (!c) return CAKF_E_ARG;
    HIP_TRY(hipMemsetAsync(c->mean, 0, (size_t)c->N * sizeof(float), c->stream));
    HIP_TRY(hipMemsetAsync(c->diag, 0, sizeof(Diag), c->stream));
    c->rank = 0;
    c->orth = 0;
    return CAKF_OK;
}

extern "C" int cakf_state(cakf_ctx* c, float** mean, float** factor, int* ld, int* rank) {
    if (!c) return CAKF_E_ARG;
    if (mean) *mean = c->mean;
    if (factor) *factor = c->M[c->cur];
    if (ld) *ld = c->ldM;
    if (rank) *rank = c->rank;
    return CAKF_OK;
}

extern "C" int cakf_copy_state(cakf_ctx* c, float* mean, float* factor, int ld) {
    if (!c || (factor && ld < c->rank)) return CAKF_E_ARG;
    if (mean)
        HIP_TRY(hipMemcpyAsync(mean, c->mean, (size_t)c->N * sizeof(float),
                               hipMemcpyDeviceToDevice, c->stream));
    if (factor && c->rank > 0)
        launch_copy_rows(c->M[c->cur], c->ldM, factor, ld, c->N, c->rank, c->stream);
    return CAKF_OK;
}

extern "C" int cakf_set_state(cakf_ctx* c, const float* mean, const float* factor, int ld,
                              int rank) {
    if (!c || !mean || rank < 0 || rank > c->Kmax || (rank > 0 && (!factor || ld < rank)))
        return CAKF_E_ARG;
    HIP_TRY(hipMemcpyAsync(c->mean, mean, (size_t)c->N * sizeof(float), hipMemcpyDeviceToDevice,
                           c->stream));
    if (rank > 0) launch_copy_rows(factor, ld, c->M[c->cur], c->ldM, c->N, rank, c->stream);
    c->rank = rank;
    c->orth = 0;
    return CAKF_OK;
}

extern "C" int cakf_predict(cakf_ctx* c) {
    if (!c) return CAKF_E_ARG;
    const float a = (float)c->cfg.ou_coeff;
    if (c->cfg.temporal == CAKF_TEMPORAL_MATERN32) {
        // A^t = a [[1 + s, s], [-s, 1 - s]], s = -log a, on each point's (value, derivative)
        const double ad = c->cfg.ou_coeff, sd = -std::log(ad);
        const float t[4] = {(float)(ad * (1.0 + sd)), (float)(ad * sd), (float)(-ad * sd),
                            (float)(ad * (1.0 - sd))};
        launch_predict_pairs(c->mean, c->M[c->cur], c->n, c->ldM, c->rank, t, c->stream);
        c->orth = 0;        // the transition mixes the value and derivative rows
    } else if (a != 1.0f) {
        launch_scale_state(c->mean, c->M[c->cur], c->n, c->ldM, c->rank, a, c->stream);
        c->orth_scale *= (double)a * (double)a;
    }
    return CAKF_OK;
}

// Fill the scalar record fields of a step without data.
__global__ void k_empty_record(double* loglik, int* n_actions) {
    if (loglik) *loglik = 0.0;
    if (n_actions) *n_actions = 0;
}

// A bounded wait of the tridiagonalisation that gave up counts as a non-finite event.
__global__ void k_note_abort(const int* abort_flag, Diag* dg) {
    if (*abort_flag) dg->nonfinite += 1;
}

__global__ void k_count_diag(const LoopState* ls, Diag* dg) {
    dg->dropped += ls->dropped;
    dg->nonfinite += ls->nonfinite;
    dg->bad_index += ls->bad_index;
    dg->steps += 1;
    dg->loglik += ls->loglik;
}

// Row-major GEMM C (M x N) = alpha op(A) op(B) + beta C through column-major rocBLAS
// (a row-major matrix is its transpose in column-major storage).
static rocblas_status sgemm_rm(rocblas_handle h, bool ta, bool tb, int M, int N, int K,
                               float alpha, const float* A, int lda, const float* B, int ldb,
                               float beta, float* C, int ldc) {
    return rocblas_sgemm(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                         ta ? rocblas_operation_transpose : rocblas_operation_none, N, M, K,
                         &alpha, B, ldb, A, lda, &beta, C, ldc);
}

// The action loop of the block-residual policy: rounds of bt actions.  A round splits the
// current residual over bt observation groups (the new action columns), multiplies them by
// the prior covariance of the observed points in one block product, subtracts the low-rank
// part (Mo^T S_round, then Mo times that), and forms all Gram columns of the round in one
// FP64-accumulated product G = S^T [U_r | S_r | V_r | r0] (rows: every action so far),
// from which the incremental Cholesky step takes one column per action.
static int block_rounds(cakf_ctx* c, const ObsDims& d, int imax, hipStream_t st) {
    const int nu2 = c->cfg.kernel, dist = c->cfg.dist, m = d.m;
    const float noise = (float)c->cfg.noise_var;
    for (int j0 = 0; j0 < imax;) {
        const int bt = std::min(c->bmax, imax - j0);
        launch_block_residual(c->U, c->V, c->S, c->r0, c->beta, noise, d, j0, bt, c->ls, st);
        launch_block_product(nu2, dist, c->cfg.prec, c->Xo, m, c->Xo, m, d.mp, c->S + j0,
                             d.imax, bt, c->Bth, c->Btl, (float)c->cfg.signal_var, c->U + j0,
                             d.imax, st, block_product_splits(m, d.mp, bt, c->bpart_elems),
                             c->bpart);
        if (d.rank > 0) {
            // T[:, j0 + g] = Mo^T s_(j0 + g)   (column-major, ld ldmo)
            launch_round_mot(c->Mo, c->S, d, j0, bt, c->bpart32, c->T, st);
            // V[:, j0 + g] = Mo T[:, j0 + g]   (row-major rows of V, ld imax)
            const float one = 1.0f, zero = 0.0f;
            BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none,
                                   bt, m, d.rank, &one, c->T + (size_t)j0 * c->ldmo, c->ldmo,
                                   c->Mo, c->ldmo, &zero, c->V + j0, d.imax));
        }
        // G = S^T [U_r | S_r | V_r | r0] over every action so far
        launch_round_gram(c->U, c->V, c->S, c->r0, d, j0, bt, c->bpart64, c->bG, c->ldz, st);
        {
            // the round's bt Cholesky steps in one launch
            PhaseTimer t(c, CAKF_PHASE_TAIL);
            TailDirect td;
            td.G = c->bG;
            td.ld = c->ldz;
            td.uc = 0;
            td.sc = bt;
            td.vc = 2 * bt;
            td.rc = 3 * bt;
            launch_tail(d, j0, c->cfg.noise_var, c->cfg.resid_tol, c->cfg.pivot_tol, c->Linv,
                        c->LinvT, c->L, c->LSinv, c->LSinvT, c->alpha, c->beta, c->ls, st, td,
                        bt);
        }
        j0 += bt;
    }
    return CAKF_OK;
}

extern "C" int cakf_update(cakf_ctx* c, const int32_t* idx, const float* y, int m,
                           const float* actions, const cakf_record* rec) {
    if (!c || m < 0 || m > c->mmax) return CAKF_E_ARG;
    const cakf_record none = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (!rec) rec = &none;
    hipStream_t st = c->stream;
    if (m == 0) {
        hipLaunchKernelGGL(k_empty_record, dim3(1), dim3(1), 0, st, rec->loglik, rec->n_actions);
        return CAKF_OK;
    }
    if (!idx || !y) return CAKF_E_ARG;
    const bool cg = c->cfg.policy == CAKF_POLICY_CG;
    const bool block = c->cfg.policy == CAKF_POLICY_BLOCK;
    if (c->cfg.policy == CAKF_POLICY_GIVEN && !actions) return CAKF_E_ARG;
    if (c->rank > c->r) return CAKF_E_STATE;
    const int imax = std::min(c->imax, m);
    ObsDims d;
    d.m = m;
    d.mp = round_up(m, SYM_TILE);
    d.imax = c->imax;
    d.rank = c->rank;
    d.ldmo = c->ldmo;
    float* M = c->M[c->cur];
    const size_t tri = (size_t)c->imax * c->imax * sizeof(double);
    HIP_TRY(hipMemsetAsync(c->ls, 0, sizeof(LoopState), st));
    HIP_TRY(hipMemsetAsync(c->Linv, 0, tri, st));
    HIP_TRY(hipMemsetAsync(c->LinvT, 0, tri, st));
    HIP_TRY(hipMemsetAsync(c->L, 0, tri, st));
    HIP_TRY(hipMemsetAsync(c->LSinv, 0, tri, st));
    HIP_TRY(hipMemsetAsync(c->LSinvT, 0, tri, st));
    HIP_TRY(hipMemsetAsync(c->alpha, 0, c->imax * sizeof(double), st));
    HIP_TRY(hipMemsetAsync(c->beta, 0, c->imax * sizeof(double), st));
    launch_gather(c->Xs, c->n, c->mean, M, c->ldM, idx, y, block ? nullptr : actions,
                  (cg || block) ? 1 : 0, d, c->Xo, c->r0, c->Mo, c->S, c->U, c->ls, st);
    if (block) {
        const int rc = block_rounds(c, d, imax, st);
        if (rc) return rc;
    } else if (d.rank > 0) {
        // t_0 = Mo^T s_0 (s_0 = r0 for CG, the first given action otherwise), column 0 of
        // T (rank x imax, column-major, ld ldmo); the later columns are formed one per
        // action, the partial sums in next_action and their FP64 sum in sym_tiles
        int nb = 0;
        launch_colsum_partial(c->Mo, c->ldmo, m, d.rank, cg ? c->r0 : c->S, cg ? 1 : c->imax,
                              c->mpart, c->ldmo, st, &nb);
        launch_colsum_final(c->mpart, c->ldmo, nb, d.rank, c->T, 1, st);
    }
    const int nu2 = c->cfg.kernel, dist = c->cfg.dist;
    const float noise = (float)c->cfg.noise_var;
    // column products of s_0
    int ncp = 0, nmpart = 0;
    if (!block)
        launch_next_action(0, 0, c->U, c->Mo, c->r0, c->S, c->V, c->T, noise, d, 0, c->mpart,
                           c->cpart, c->gs, c->ls, nullptr, st, &ncp);
    TriArgs ta;
    ta.Linv = c->Linv;
    ta.LinvT = c->LinvT;
    ta.alpha = c->alpha;
    ta.tri = c->tri;
    ta.ctr = c->ctr;
    ta.ttpart = c->ttpart;
    ta.noise_var = c->cfg.noise_var;
    // beta after action j lives in bbuf[j & 1]
    double* bbuf[2] = {c->beta, c->beta2};
    TailArgs tl;
    tl.imax = d.imax;
    tl.tri = c->tri;
    tl.colvec = c->colvec;
    tl.fupart = c->fupart;
    tl.Linv = c->Linv;
    tl.LinvT = c->LinvT;
    tl.L = c->L;
    tl.alpha = c->alpha;
    tl.SS = c->SS;
    tl.noise_var = c->cfg.noise_var;
    tl.resid_tol = c->cfg.resid_tol;
    tl.pivot_tol = c->cfg.pivot_tol;
    for (int j = 0; j < (block ? 0 : imax); ++j) {
        {
            KernelTimer t(c, CAKF_PHASE_SYM_TILES);
            launch_sym_tiles(nu2, dist, c->cfg.prec != CAKF_PREC_FP32, c->Xo, c->S, d, j,
                             c->part, (j > 0 && d.rank > 0) ? c->mpart : nullptr, nmpart,
                             c->T, c->cpart, ncp, c->gs, c->colvec, c->ls, ta, st, t.start,
                             t.stop);
        }
        int nfu = 0;
        {
            PhaseTimer t(c, CAKF_PHASE_FORM_U);
            launch_form_u(c->part, c->S, c->U, d, j, c->cfg.signal_var, c->fupart, c->ls, st,
                          &nfu);
        }
        tl.nfu = nfu;
        tl.beta_in = bbuf[(j + 1) & 1];
        tl.beta_out = bbuf[j & 1];
        if (j + 1 < imax) {
            // the rest of action j's Cholesky step, then action j + 1
            PhaseTimer t(c, CAKF_PHASE_NEXT_ACTION);
            launch_next_action(cg ? 1 : 0, 1, c->U, c->Mo, c->r0, c->S, c->V, c->T, noise, d,
                               j + 1, c->mpart, c->cpart, c->gs, c->ls, &tl, st, &ncp);
            nmpart = ncp;
        } else {
            PhaseTimer t(c, CAKF_PHASE_TAIL);
            launch_tail_final(tl, j, c->beta2, c->beta, c->SSwork, c->ls, st);
        }
    }
    launch_build_block(c->S, c->LinvT, c->beta, d, c->B, c->bp, c->bp, rec->W_obs, rec->w_obs,
                       rec->S, c->ls, st);
    const int b = c->imax + 1;
    if (d.rank > 0) {
        const float one = 1.0f, zero = 0.0f;
        // Q^T = B^T Mo  (b x rank, column-major ld bp), so that the product with the factor
        // below needs no transposed operand (the library's kernel for that form is about
        // twice as fast at these shapes)
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_transpose, b,
                               d.rank, m, &one, c->B, c->bp, c->Mo, c->ldmo, &zero, c->Q, c->bp));
    }
    // Y = Sigma[:, idx] B into the new columns rank .. rank + b of the factor
    {
        PhaseTimer t(c, CAKF_PHASE_BLOCK_PRODUCT);
        // the mean column w (column imax) is summed in FP32 in the BF16 modes: the mean
        // increment is a small difference of the two parts of P^- H^T w
        launch_block_product(nu2, dist, c->cfg.prec, c->Xs, c->n, c->Xo, m, d.mp, c->B, c->bp, b,
                             c->Bth, c->Btl, (float)c->cfg.signal_var, M + d.rank, c->ldM, st,
                             block_product_splits(c->n, d.mp, b, c->bpart_elems), c->bpart,
                             c->imax);
    }
    // the scaled-derivative rows of Sigma_inf H^T [W w] are zero (I_2 (x) Sigma)
    if (c->N > c->n) launch_zero_cols(M + (size_t)c->n * c->ldM + d.rank, c->ldM, c->N - c->n, b, st);
    if (d.rank > 0) {
        const float mone = -1.0f, one = 1.0f;
        // Y -= M^- Q  (the low-rank part of P^- H^T [W w]); column-major: Y^T -= Q^T M^-^T
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_none, b, c->N,
                               d.rank, &mone, c->Q, c->bp, M, c->ldM, &one, M + d.rank, c->ldM));
    }
    launch_mean_add(c->mean, M, c->N, c->ldM, d.rank + c->imax, st);
    launch_finish_record(c->ls, c->L, c->Linv, c->imax, rec->chol, rec->chol_inv, rec->loglik,
                         rec->n_actions, st);
    hipLaunchKernelGGL(k_count_diag, dim3(1), dim3(1), 0, st, c->ls, c->diag);
    c->rank += c->imax;
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

// Device memory the truncation works in: the FP64 Gram (its buffer then holds the
// tridiagonal's eigenvectors), the Gram's slab partials, the tridiagonalisation's
// reflectors, tau, exchange vectors and barrier words, the tridiagonal (d, e), the
// solver's info word and V_r.
struct TruncWork {
    double* G;
    double* gwork;
    size_t gwork_elems;
    double *tdV, *tdtau, *tdp, *tdrow;   // tdV == nullptr: no one-launch tridiagonalisation
    unsigned* tdctr;
    int* tdabort;
    double *eigval, *offdiag;
    int* info;
    float* Vr;
};

static TruncWork context_work(cakf_ctx* c) {
    return TruncWork{c->G, c->gwork, c->gram_work_elems, c->tdV, c->tdtau, c->tdp, c->tdrow,
                     c->tdctr, c->tdabort, c->eigval, c->offdiag, c->info, c->Vr};
}

// Replace the rows x K factor M (row-major, ld) by M V_r in Mout (ld ldo), V_r the leading
// r eigenvectors of M^T M (FP64 Gram, FP64 symmetric eigensolver, FP32 rotation).  With
// lam, the first orth columns of M are known to be orthogonal with squared norms
// orth_scale * lam (their Gram block is not computed), and lam receives the r kept
// eigenvalues in descending order, the squared norms of the columns of Mout.
static int truncate_factor(cakf_ctx* c, const TruncWork& w, const float* M, int rows, int ld,
                           int K, int r, float* Mout, int ldo, double* rotation, int orth = 0,
                           double orth_scale = 1.0, double* lam = nullptr) {
    hipStream_t st = c->stream;
    {
        PhaseTimer t(c, CAKF_PHASE_GRAM);
        launch_gram64(M, rows, ld, K, w.G, w.gwork, w.gwork_elems, st, orth, lam, orth_scale);
    }
    bool picked = false;
    {
        PhaseTimer t(c, CAKF_PHASE_EIG);
        // G = Q T Q^T in one cooperative launch, the r leading eigenpairs of T (bisection,
        // twisted factorisation, clusters by inverse iteration), back-transformed into V_r
        // directly.  Larger K, or a device that cannot co-schedule the launch, takes the
        // library's dense solver.
        // work area of the Gram's partial sums (consumed by now): Z, Z X, E, E^2, lam
        const size_t need = 2 * (size_t)K * r + 2 * (size_t)r * r + tri_eigen_work_elems(K, r);
        if (w.tdV && K >= 3 && K <= TD_MAXK && K <= tri_eigen_max_k() && need <= w.gwork_elems) {
            if (launch_tridiag(w.G, K, w.tdV, w.tdtau, w.eigval, w.offdiag, w.tdp, w.tdrow,
                               w.tdctr, w.tdabort, st) == hipSuccess) {
                hipLaunchKernelGGL(k_note_abort, dim3(1), dim3(1), 0, st, w.tdabort, c->diag);
                double* Zr = w.gwork;                       // K x r row-major = Z^T col-major
                double* Zx = Zr + (size_t)K * r;
                double* E = Zx + (size_t)K * r;
                double* E2 = E + (size_t)r * r;
                launch_tri_eigen(w.eigval, w.offdiag, K, r, E2 + (size_t)r * r, Zr, st);
                // symmetric orthogonalisation Z X, X = I - E/2 + 3/8 E^2, E = Z^T Z - I: the
                // twisted vectors of closely spaced eigenvalues are orthogonal only to about
                // eps ||T|| / gap; mixing within the kept subspace leaves M V_r V_r^T M^T as
                // it is.  Column-major: Zt = Z^T (r x K, ld r), E = Zt Zt^T, Zt X = (Z X)^T.
                const double one = 1.0, zero = 0.0;
                BLAS_TRY(rocblas_dgemm(c->blas, rocblas_operation_none,
                                       rocblas_operation_transpose, r, r, K, &one, Zr, r, Zr,
                                       r, &zero, E, r));
                launch_lowdin(E, E2, r, 0, st);
                BLAS_TRY(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none,
                                       r, r, r, &one, E, r, E, r, &zero, E2, r));
                launch_lowdin(E, E2, r, 1, st);
                BLAS_TRY(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none,
                                       r, K, r, &one, E2, r, Zr, r, &zero, Zx, r));
                launch_backtransform(Zx, r, 1, w.tdV, w.tdtau, K, r, w.Vr, rotation, st);
                if (lam) launch_store_lam(E2 + (size_t)r * r, K, r, 0, lam, st);
                picked = true;
            } else {
                (void)hipGetLastError();
            }
        }
        if (!picked) {
            BLAS_TRY(rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_lower, K,
                                      w.G, K, w.eigval, w.offdiag, w.info));
            if (lam) launch_store_lam(w.eigval, K, r, 1, lam, st);
        }
    }
    {
        PhaseTimer t(c, CAKF_PHASE_ROTATE);
        if (!picked) launch_pick_rotation(w.G, K, r, w.Vr, rotation, st);
        const float one = 1.0f, zero = 0.0f;
        // Mout (row-major n x r) = M V_r: column-major (r x n) = V_r^T (r x K) M^T (K x n),
        // V_r row-major K x r being V_r^T column-major (no transposed operand)
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_none, r, rows,
                               K, &one, w.Vr, r, M, ld, &zero, Mout, ldo));
    }
    return CAKF_OK;
}

extern "C" int cakf_truncate(cakf_ctx* c, double* rotation) {
    if (!c) return CAKF_E_ARG;
    const int K = c->rank;
    if (K <= c->r) return CAKF_OK;
    int rc = truncate_factor(c, context_work(c), c->M[c->cur], c->N, c->ldM, K, c->r,
                             c->M[1 - c->cur], c->ldM, rotation, c->orth, c->orth_scale,
                             c->lam);
    if (rc) return rc;
    c->cur = 1 - c->cur;
    c->rank = c->r;
    c->orth = c->r;
    c->orth_scale = 1.0;
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

// ------------------------------------------------------- log-likelihood derivative
extern "C" int cakf_loglik_grad(cakf_ctx* c, int T, const cakf_tape_step* tape, double dt,
                                double* grad) {
    if (!c || !grad || T < 1 || !tape || !c->gMb[0] || !(dt >= 0)) return CAKF_E_ARG;
    hipStream_t st = c->stream;
    const int n = c->n, imax = c->imax, bp = c->bp, ldM = c->ldM, ldmo = c->ldmo;
    const int I1 = imax + 1;
    const double ell = c->cfg.lengthscale, s2 = c->cfg.signal_var;
    const float a = (float)c->cfg.ou_coeff;
    // host-side shapes of every step (ranks follow from the update and truncation rules)
    std::vector<int> kept(T, 0);
    for (int k = 0; k < T; ++k) {
        const cakf_tape_step& t = tape[k];
        if (t.m < 0 || t.m > c->mmax || !t.mean || !t.factor || t.rank < 0 ||
            t.rank > c->r || (t.rank > 0 && t.ld < t.rank))
            return CAKF_E_ARG;
        if (t.m > 0 && (!t.idx || !t.y || !t.S || !t.W_obs || !t.w_obs || !t.chol ||
                        !t.chol_inv || !t.n_actions))
            return CAKF_E_ARG;
        const int prev = k > 0 ? tape[k - 1].rank : 0;
        const int full = t.m > 0 ? prev + imax : prev;
        if (t.rotation ? (t.rank_full != full || t.rank > full) : t.rank != full)
            return CAKF_E_ARG;
        if (t.m > 0) HIP_TRY(hipMemcpyAsync(&kept[k], t.n_actions, sizeof(int),
                                            hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemsetAsync(c->gacc, 0, 4 * sizeof(double), st));
    HIP_TRY(hipMemsetAsync(c->gmb, 0, (size_t)n * sizeof(float), st));
    HIP_TRY(hipMemsetAsync(c->gMb[0], 0, (size_t)n * ldM * sizeof(float), st));
    int cur = 0;   // gMb[cur] holds the adjoint of the factor passed on by step k
    const int nu2 = c->cfg.kernel, dist = c->cfg.dist;
    for (int k = T - 1; k >= 0; --k) {
        const cakf_tape_step& t = tape[k];
        const int rank = k > 0 ? tape[k - 1].rank : 0;     // columns of M^+_{k-1}
        const float* mprev = k > 0 ? tape[k - 1].mean : nullptr;
        const float* Mprev = k > 0 ? tape[k - 1].factor : nullptr;
        const int ldprev = k > 0 ? tape[k - 1].ld : 1;
        // 1. truncation: Mbar_k = Mbar^+_k V_r^T
        float* Mbk = c->gMb[cur];
        if (t.rotation) {
            const int K = t.rank_full;
            // V_r^T (t.rank x K, FP32), so that the product has no transposed operand
            launch_to_f32_t(t.rotation, K, t.rank, c->Vr, st);
            Mbk = c->gMb[1 - cur];
            if (K > 0)
                BLAS_TRY(sgemm_rm(c->blas, false, false, n, K, t.rank, 1.0f, c->gMb[cur], ldM,
                                  c->Vr, K, 0.0f, Mbk, ldM));
            cur = 1 - cur;
        }
        const int J = t.m > 0 ? kept[k] : 0;
        if (J > 0) {
            const int m = t.m, mp = round_up(m, 32);
            // 2. Ybar, B, Mo, r0 and the FP64 copies
            launch_adj_pack_ybar(Mbk, ldM, rank, imax, c->gmb, n, c->gYb, bp, st);
            launch_adj_obs_prep(c->Xs, n, t.idx, t.y, m, mp, a, mprev, Mprev, ldprev, rank,
                                t.W_obs, t.w_obs, t.S, imax, bp, ldmo, c->Xo, c->Mo, c->gBq,
                                c->gW64, c->gSr64, st);
            // 3. Bbar = sigma_f2 K(Xo, X) Ybar and the kernel terms of Y
            {
                int gx, gy, rps, gx2, gy2, rps2;
                adj_tiles_geometry(n, m, &gx, &gy, &rps);
                adj_tiles_geometry(m, m, &gx2, &gy2, &rps2);
                if ((size_t)gy * mp * bp > c->gbpart_elems ||
                    gx * gy * adj_tiles_launches(imax + 1) > c->gspart_blocks ||
                    gx2 * gy2 * adj_tiles_launches(imax) > c->gspart_blocks)
                    return CAKF_E_ARG;
            }
            int nblk = 0;
            const int ns = launch_adj_tiles(nu2, dist, true, c->Xs, n, c->gYb, bp, c->Xo, m,
                                            c->gBq, bp, imax + 1, c->gbpart, bp,
                                            (size_t)mp * bp, c->gspart, &nblk, st);
            if (ns < 0 || (size_t)ns * mp * bp > c->gbpart_elems || nblk > c->gspart_blocks)
                return CAKF_E_ARG;
            launch_adj_bbar_reduce(c->gbpart, (size_t)mp * bp, bp, ns, m, mp, imax + 1,
                                   (float)s2, c->gBb, bp, st);
            launch_adj_scalars(c->gspart, nblk, 1.0, s2 / ell, c->gacc, 2, 0, st);
            if (rank > 0) {
                // Q = Mo^T B, T = Mo^T S, Qbar = -a M^+_{k-1}^T Ybar
                BLAS_TRY(sgemm_rm(c->blas, true, false, rank, bp, m, 1.0f, c->Mo, ldmo, c->gBq,
                                  bp, 0.0f, c->Q, bp));
                BLAS_TRY(sgemm_rm(c->blas, true, false, rank, imax, m, 1.0f, c->Mo, ldmo, t.S,
                                  imax, 0.0f, c->T, imax));
                BLAS_TRY(sgemm_rm(c->blas, true, false, rank, bp, n, -a, Mprev, ldprev, c->gYb,
                                  bp, 0.0f, c->gQb, bp));
                // Mbar^- -= Ybar Q^T;  Bbar += Mo Qbar;  Mobar = B Qbar^T
                BLAS_TRY(sgemm_rm(c->blas, false, true, n, rank, bp, -1.0f, c->gYb, bp, c->Q,
                                  bp, 1.0f, Mbk, ldM));
                BLAS_TRY(sgemm_rm(c->blas, false, false, m, bp, rank, 1.0f, c->Mo, ldmo,
                                  c->gQb, bp, 1.0f, c->gBb, bp));
                BLAS_TRY(sgemm_rm(c->blas, false, true, m, rank, bp, 1.0f, c->gBq, bp, c->gQb,
                                  bp, 0.0f, c->gMob, ldmo));
            }
            // 4. the Cholesky form in FP64: G1 = W^T Bbar, G2 = S^T [S r0]
            launch_to_f64(c->gBb, bp, m, I1, c->gBb64, I1, st);
            // (slab products: the library's GEMM does not split the m-long inner dimension)
            launch_atb64(c->gW64, imax, c->gBb64, I1, m, imax, I1, c->gatb, c->gG1, I1, st);
            launch_atb64(c->gSr64, I1, c->gSr64, I1, m, imax, I1, c->gatb, c->gG2, I1, st);
            launch_adj_small(J, imax, c->gG1, c->gG2, t.chol, t.chol_inv, c->gX1, c->gX2,
                             c->gCc, c->gacc, 3, st);
            // 5. [Z rbar0] = S [Cbar cbar]; the kernel terms of C = S^T Ghat S
            BLAS_TRY(sgemm_rm(c->blas, false, false, m, I1, imax, 1.0f, t.S, imax, c->gCc, I1,
                              0.0f, c->gZr, I1));
            int nblk2 = 0;
            if (launch_adj_tiles(nu2, dist, false, c->Xo, m, c->gZr, I1, c->Xo, m, t.S, imax, J,
                                 nullptr, 0, 0, c->gspart, &nblk2, st) < 0 ||
                nblk2 > c->gspart_blocks)
                return CAKF_E_ARG;
            launch_adj_scalars(c->gspart, nblk2, 1.0, s2 / ell, c->gacc, 2, 0, st);
            if (rank > 0)
                BLAS_TRY(sgemm_rm(c->blas, false, true, m, rank, imax, -2.0f, c->gZr, I1, c->T,
                                  imax, 1.0f, c->gMob, ldmo));
            // 6. scatter Mobar and -rbar0 into the adjoints of M^-, m^-
            launch_adj_scatter(t.idx, m, n, c->gMob, ldmo, rank, c->gZr, I1, imax, Mbk, ldM,
                               c->gmb, st);
        }
        // 7. predict: d/da and the adjoints of step k-1 (Mbar^- lives in Mbk's first columns)
        if (k > 0) {
            const int nb = launch_adj_predict(c->gmb, mprev, Mbk, ldM, Mprev, ldprev, rank, n,
                                              a, c->gpart, st);
            launch_sum_into(c->gpart, nb, c->gacc, 1, st);
        }
    }
    HIP_TRY(hipMemcpyAsync(grad, c->gacc, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (dt > 0) {
        // a = exp(-dt / ell_t):  da / dell_t = a dt / ell_t^2 = a (log a)^2 / dt
        const double la = std::log(c->cfg.ou_coeff);
        grad[1] *= c->cfg.ou_coeff * la * la / dt;
    }
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

// ---------------------------------------------------------------- smoother (Alg. 3)
extern "C" int cakf_smooth_begin(cakf_ctx* c, const int32_t* idx, const float* w_obs,
                                 const float* W_obs, int m) {
    if (!c || !c->Xp || m < 0 || m > c->mmax) return CAKF_E_ARG;
    if (m > 0 && (!idx || !w_obs || !W_obs)) return CAKF_E_ARG;
    hipStream_t st = c->stream;
    c->sm_cur = 0;
    // ws_T = H^T w_obs, Ws_T = H^T W_obs (no earlier smoother messages: rs = 0, Bs = 0)
    HIP_TRY(hipMemsetAsync(c->sm_B, 0, (size_t)c->np * c->bps * sizeof(float), st));
    launch_smooth_messages(c->sm_B, c->bps, c->n, idx, m, m > 0 ? c->imax : 0, 0, w_obs, W_obs,
                           c->imax, nullptr, 0, c->sm_ws, c->sm_W[0], c->ldWs, st);
    c->sm_rank = m > 0 ? c->imax : 0;
    c->sm_started = true;
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

static int smooth_input_ok(const cakf_ctx* c, const cakf_smooth_input* in) {
    if (!in || !in->mean) return 0;
    if (in->rank < 0 || in->rank > c->Kmax || (in->rank > 0 && (!in->factor || in->ld < in->rank)))
        return 0;
    if (in->pred_rank < 0 || in->pred_rank > c->Kmax ||
        (in->pred_rank > 0 && (!in->pred_factor || in->pred_ld < in->pred_rank)))
        return 0;
    if (in->m < 0 || in->m > c->mmax || (in->m > 0 && (!in->idx || !in->w_obs || !in->W_obs)))
        return 0;
    return 1;
}

// Smoothed moments from the filter moments (mean, factor) scaled by g and the current
// messages [ws Ws] propagated by ar:  Bs = ar [ws Ws],  Y = Sigma Bs,
// Z = Y - g^2 M (M^T Bs),  mean_out = g m + Z[:, 0],  factor_out = [g M | Z[:, 1:]].
// Leaves Bs in sm_B and Y in sm_Y.
static int smooth_moments(cakf_ctx* c, const cakf_smooth_input* in, float g, float ar,
                          float* mean_out, float* factor_out, int ld_out, float* var_out) {
    const int rs = c->sm_rank;
    const int b = 1 + rs;
    hipStream_t st = c->stream;
    const float one = 1.0f, zero = 0.0f, mg2 = -g * g;
    float* Ws = c->sm_W[c->sm_cur];
    // Bs = ar [ws Ws]
    launch_smooth_pack(c->sm_ws, Ws, c->ldWs, c->n, c->np, rs, ar, c->sm_B, c->bps, st);
    // Y = Sigma Bs (kernel matrix over all points, never stored)
    {
        PhaseTimer t(c, CAKF_PHASE_BLOCK_PRODUCT);
        launch_block_product(c->cfg.kernel, c->cfg.dist, c->cfg.prec, c->Xs, c->n, c->Xp, c->n,
                             c->np, c->sm_B, c->bps, b, c->sm_Bth, c->sm_Btl,
                             (float)c->cfg.signal_var, c->sm_Y, c->bps, st,
                             block_product_splits(c->n, c->np, b, c->bpart_elems), c->bpart,
                             0);    // the mean message ws in FP32 (BF16 modes)
    }
    // Z = Y - g^2 M (M^T Bs)
    HIP_TRY(hipMemcpyAsync(c->sm_Z, c->sm_Y, (size_t)c->n * c->bps * sizeof(float),
                           hipMemcpyDeviceToDevice, st));
    if (in->rank > 0) {
        // Q^T = Bs^T M (b x rank, column-major ld bps), then Z^T -= g^2 Q^T M^T: neither
        // product has a transposed operand on the long side
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_transpose, b,
                               in->rank, c->n, &one, c->sm_B, c->bps, in->factor, in->ld, &zero,
                               c->sm_Q, c->bps));
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_none, b, c->n,
                               in->rank, &mg2, c->sm_Q, c->bps, in->factor, in->ld, &one,
                               c->sm_Z, c->bps));
    }
    launch_smooth_out(in->mean, in->factor, in->ld, in->rank, g, c->sm_Z, c->bps, b, c->n,
                      (float)c->cfg.signal_var, mean_out, factor_out, ld_out, var_out, st);
    return CAKF_OK;
}

extern "C" int cakf_smooth_step(cakf_ctx* c, const cakf_smooth_input* in, float* mean_out,
                                float* factor_out, int ld_out, float* var_out, int* out_rank) {
    if (!c || !c->sm_started || !smooth_input_ok(c, in)) return CAKF_E_ARG;
    const int rs = c->sm_rank;
    const int b = 1 + rs;
    if (factor_out && ld_out < in->rank + rs) return CAKF_E_ARG;
    hipStream_t st = c->stream;
    const float one = 1.0f, zero = 0.0f, mone = -1.0f;
    float* Ws = c->sm_W[c->sm_cur];
    int rc = smooth_moments(c, in, 1.0f, (float)c->cfg.ou_coeff, mean_out, factor_out, ld_out,
                            var_out);
    if (rc) return rc;
    if (out_rank) *out_rank = in->rank + rs;
    // Pm = P_k^- A^T [ws Ws] = Y - M_k^- (M_k^-^T Bs), reusing Z
    const int i = in->m > 0 ? c->imax : 0;
    if (in->m > 0) {
        HIP_TRY(hipMemcpyAsync(c->sm_Z, c->sm_Y, (size_t)c->n * c->bps * sizeof(float),
                               hipMemcpyDeviceToDevice, st));
        if (in->pred_rank > 0) {
            BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_transpose,
                                   b, in->pred_rank, c->n, &one, c->sm_B, c->bps,
                                   in->pred_factor, in->pred_ld, &zero, c->sm_Q, c->bps));
            BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_none, b,
                                   c->n, in->pred_rank, &mone, c->sm_Q, c->bps, in->pred_factor,
                                   in->pred_ld, &one, c->sm_Z, c->bps));
        }
        // R = W_obs^T Pm[idx, :] (imax x b), WR = W_obs R (m x b); R is kept as R^T
        // (b x imax, column-major ld bps) so that WR^T = R^T W_obs^T needs no transpose
        launch_gather_rows(c->sm_Z, c->bps, in->idx, in->m, c->n, b, c->sm_Gr, c->bps, st);
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_transpose, b,
                               c->imax, in->m, &one, c->sm_Gr, c->bps, in->W_obs, c->imax, &zero,
                               c->sm_R, c->bps));
        BLAS_TRY(rocblas_sgemm(c->blas, rocblas_operation_none, rocblas_operation_none, b, in->m,
                               c->imax, &one, c->sm_R, c->bps, in->W_obs, c->imax, &zero,
                               c->sm_WR, c->bps));
    }
    // ws = w + proj[:, 0], [W, proj[:, 1:]] with proj = Bs - H^T (W_obs R)
    float* Wn = c->sm_W[1 - c->sm_cur];
    launch_smooth_messages(c->sm_B, c->bps, c->n, in->idx, in->m, i, rs, in->w_obs, in->W_obs,
                           c->imax, in->m > 0 ? c->sm_WR : nullptr, c->bps, c->sm_ws, Wn,
                           c->ldWs, st);
    const int K = i + rs;
    if (K > c->r) {
        int rc = truncate_factor(c, context_work(c), Wn, c->n, c->ldWs, K, c->r, Ws, c->ldWs,
                                 nullptr);
        if (rc) return rc;
        c->sm_rank = c->r;          // result landed in the current buffer
    } else {
        c->sm_cur = 1 - c->sm_cur;
        c->sm_rank = K;
    }
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

extern "C" int cakf_smooth(cakf_ctx* c, int T, const cakf_smooth_input* steps,
                           float* mean_out, float* var_out) {
    if (!c || !c->Xp || T < 1 || !steps) return CAKF_E_ARG;
    const cakf_smooth_input& last = steps[T - 1];
    if (!last.mean || last.rank < 0 || last.rank > c->Kmax ||
        (last.rank > 0 && (!last.factor || last.ld < last.rank)))
        return CAKF_E_ARG;
    for (int k = 0; k + 1 < T; ++k)
        if (!smooth_input_ok(c, &steps[k])) return CAKF_E_ARG;
    const size_t n = c->n;
    int rc = cakf_smooth_begin(c, last.idx, last.w_obs, last.W_obs, last.m);
    if (rc) return rc;
    // step T: the filter's moments
    if (mean_out)
        HIP_TRY(hipMemcpyAsync(mean_out + (T - 1) * n, last.mean, n * sizeof(float),
                               hipMemcpyDeviceToDevice, c->stream));
    if (var_out)
        launch_marginal_var(last.factor, c->n, last.ld, last.rank, (float)c->cfg.signal_var,
                            nullptr, c->n, var_out + (T - 1) * n, c->stream);
    for (int k = T - 2; k >= 0; --k) {
        rc = cakf_smooth_step(c, &steps[k], mean_out ? mean_out + k * n : nullptr, nullptr, 0,
                              var_out ? var_out + k * n : nullptr, nullptr);
        if (rc) return rc;
    }
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

extern "C" int cakf_interpolate(cakf_ctx* c, const cakf_smooth_input* in, double a_left,
                                double a_right, int smoothed, float* mean_out,
                                float* factor_out, int ld_out, float* var_out, int* out_rank) {
    if (!c || !smooth_input_ok(c, in)) return CAKF_E_ARG;
    if (!(a_left > 0.0) || a_left > 1.0 || !(a_right > 0.0) || a_right > 1.0) return CAKF_E_ARG;
    if (smoothed && (!c->sm_started || !c->Xp)) return CAKF_E_ARG;
    const int rs = smoothed ? c->sm_rank : 0;
    if (factor_out && ld_out < in->rank + rs) return CAKF_E_ARG;
    const float g = (float)a_left;
    if (smoothed) {
        int rc = smooth_moments(c, in, g, (float)a_right, mean_out, factor_out, ld_out, var_out);
        if (rc) return rc;
    } else {
        launch_smooth_out(in->mean, in->factor, in->ld, in->rank, g, nullptr, 0, 1, c->n,
                          (float)c->cfg.signal_var, mean_out, factor_out, ld_out, var_out,
                          c->stream);
    }
    if (out_rank) *out_rank = in->rank + rs;
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

// ---------------------------------------------------------- path sampler (App. C)
static int sample_input_ok(const cakf_ctx* c, const cakf_sample_input* in, bool need_record) {
    if (!in || in->m < 0 || in->m > c->mmax) return 0;
    if (in->m > 0 && (!in->idx || !in->W_obs)) return 0;
    if (in->m > 0 && need_record && (!in->y || !in->S || !in->chol_inv)) return 0;
    if (in->pred_rank < 0 || in->pred_rank > c->Kmax ||
        (in->pred_rank > 0 && (!in->pred_factor || in->pred_ld < in->pred_rank)))
        return 0;
    return 1;
}

// Workspace of one forward sampler step (sizes for bsp = ns rounded to 32 columns).
struct SampleWork {
    float *B, *W, *Y, *D, *R, *Z, *Q;
    __bf16 *Bth, *Btl;
    float4* Xo;
    float* part;            // partial products of an observation-split block product
    size_t part_elems;
};

// Forward step of the sampler on the workspace w: x^- = a x_{k-1} + q, then
// x = x^- + P^- H^T W_obs L^{-1} S^T (y - x^-[idx] - sigma e).  Padding rows of the
// block-product operand are cleared by a kernel (no memset node), so the same sequence
// serves the static-scratch entry point.
static int sample_forward_impl(cakf_ctx* c, int ns, const float* x_prev, const float* q,
                               const float* e, const cakf_sample_input* in, float* x_out,
                               float* w_obs_out, const SampleWork& w) {
    hipStream_t st = c->stream;
    const int n = c->n, m = in->m, imax = c->imax, bsp = round_up(ns, 32);
    // x^- = a x_{k-1} + q
    launch_sample_predict(x_prev, q, (float)c->cfg.ou_coeff, n, ns, ns, x_out, st);
    if (m == 0) return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
    const int mp = round_up(m, SYM_TILE);
    // d = y - x^-[idx] - sigma e;  z = L^{-1} S^T d;  wobs = W_obs z (zero padding rows)
    launch_sample_innov(in->y, in->idx, x_out, ns, e, ns, (float)std::sqrt(c->cfg.noise_var), n,
                        m, ns, w.D, bsp, st);
    BLAS_TRY(sgemm_rm(c->blas, true, false, imax, ns, m, 1.0f, in->S, imax, w.D, bsp, 0.0f,
                      w.R, bsp));
    launch_sample_solve(in->chol_inv, imax, w.R, ns, bsp, w.Z, st);
    launch_fill_zero(w.B, (size_t)mp * bsp, st);
    BLAS_TRY(sgemm_rm(c->blas, false, false, m, ns, imax, 1.0f, in->W_obs, imax, w.Z, bsp,
                      0.0f, w.B, bsp));
    launch_copy_rows(w.B, bsp, w_obs_out, ns, m, ns, st);
    // x = x^- + sigma_f2 K(X, Xo) wobs - M^- (M^-^T H^T wobs)
    launch_gather_points(c->Xs, n, in->idx, m, mp, w.Xo, st);
    launch_block_product(c->cfg.kernel, c->cfg.dist, c->cfg.prec, c->Xs, n, w.Xo, m, mp,
                         w.B, bsp, ns, w.Bth, w.Btl, (float)c->cfg.signal_var,
                         w.Y, bsp, st, block_product_splits(n, mp, ns, w.part_elems), w.part);
    launch_add_cols(w.Y, bsp, n, ns, x_out, ns, st);
    if (in->pred_rank > 0) {
        launch_fill_zero(w.W, (size_t)n * bsp, st);
        launch_sample_scatter(in->idx, n, m, ns, w.B, bsp, nullptr, 0, w.W, bsp, st);
        BLAS_TRY(sgemm_rm(c->blas, true, false, in->pred_rank, ns, n, 1.0f, in->pred_factor,
                          in->pred_ld, w.W, bsp, 0.0f, w.Q, bsp));
        BLAS_TRY(sgemm_rm(c->blas, false, false, n, ns, in->pred_rank, -1.0f, in->pred_factor,
                          in->pred_ld, w.Q, bsp, 1.0f, x_out, ns));
    }
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

static int sample_forward_args_ok(const cakf_ctx* c, int ns, const float* x_prev,
                                  const float* q, const float* e, const cakf_sample_input* in,
                                  const float* x_out, const float* w_obs_out) {
    if (!c || ns < 1 || !x_prev || !q || !x_out) return 0;
    if (!sample_input_ok(c, in, true)) return 0;
    if (in->m > 0 && (!e || !w_obs_out)) return 0;
    return 1;
}

extern "C" int cakf_sample_forward(cakf_ctx* c, int ns, const float* x_prev, const float* q,
                                   const float* e, const cakf_sample_input* in, float* x_out,
                                   float* w_obs_out) {
    if (!sample_forward_args_ok(c, ns, x_prev, q, e, in, x_out, w_obs_out)) return CAKF_E_ARG;
    if (!c->sp_B || ns > c->sp_ns) return CAKF_E_ARG;
    SampleWork w{c->sp_B, c->sp_W, c->sp_Y, c->sp_D, c->sp_R, c->sp_Z, c->sp_Q,
                 c->sp_Bth, c->sp_Btl, c->sp_Xo, c->bpart, c->bpart_elems};
    return sample_forward_impl(c, ns, x_prev, q, e, in, x_out, w_obs_out, w);
}

extern "C" int cakf_sample_forward_static(cakf_ctx* c, int ns, const float* x_prev,
                                          const float* q, const float* e,
                                          const cakf_sample_input* in, float* x_out,
                                          float* w_obs_out) {
    if (!sample_forward_args_ok(c, ns, x_prev, q, e, in, x_out, w_obs_out)) return CAKF_E_ARG;
    if (ns > CAKF_STATIC_MAX_PATHS) return CAKF_E_ARG;
    void* base = scratch_of(c->device);
    if (!base) return CAKF_E_HIP;
    SampleWork w{};
    if (in->m > 0) {
        // the layout is checked against the array's size before anything is enqueued
        const size_t bsp = round_up(ns, 32), mp = round_up(in->m, SYM_TILE), n = c->n;
        Carve cv{static_cast<char*>(base), CAKF_STATIC_SCRATCH_BYTES};
        w.D = cv.take<float>(mp * bsp);
        w.R = cv.take<float>((size_t)c->imax * bsp);
        w.Z = cv.take<float>((size_t)c->imax * bsp);
        w.B = cv.take<float>(mp * bsp);
        w.Xo = cv.take<float4>(mp);
        w.Bth = cv.take<__bf16>(mp * bsp);
        w.Btl = cv.take<__bf16>(mp * bsp);
        w.Y = cv.take<float>(n * bsp);
        if (in->pred_rank > 0) {
            w.W = cv.take<float>(n * bsp);
            w.Q = cv.take<float>((size_t)in->pred_rank * bsp);
        }
        if (!cv.ok) return CAKF_E_SCRATCH;
        // what is left holds the partial products of an observation-split block product,
        // capped as in a context's workspace
        const size_t left = (cv.cap - cv.used) / sizeof(float);
        w.part_elems = std::min(left, (size_t)32 << 20);
        w.part = w.part_elems ? cv.take<float>(w.part_elems) : nullptr;
    }
    return sample_forward_impl(c, ns, x_prev, q, e, in, x_out, w_obs_out, w);
}

extern "C" int cakf_sample_lift(cakf_ctx* c, int ns, const int32_t* idx, const float* w_obs,
                                int m, float* ws_out) {
    if (!c || !c->sp_B || ns < 1 || ns > c->sp_ns || !ws_out || m < 0 || m > c->mmax)
        return CAKF_E_ARG;
    if (m > 0 && (!idx || !w_obs)) return CAKF_E_ARG;
    hipStream_t st = c->stream;
    HIP_TRY(hipMemsetAsync(ws_out, 0, (size_t)c->n * ns * sizeof(float), st));
    launch_sample_scatter(idx, c->n, m, ns, w_obs, ns, nullptr, 0, ws_out, ns, st);
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

extern "C" int cakf_sample_backward(cakf_ctx* c, int ns, const float* x, const float* factor,
                                    int ld, int rank, const cakf_sample_input* in,
                                    const float* w_obs, const float* ws_next, float* xs_out,
                                    float* ws_out) {
    if (!c || !c->sp_B || ns < 1 || ns > c->sp_ns || !x || !ws_next || !xs_out || !ws_out)
        return CAKF_E_ARG;
    if (rank < 0 || rank > c->Kmax || (rank > 0 && (!factor || ld < rank))) return CAKF_E_ARG;
    if (!sample_input_ok(c, in, false)) return CAKF_E_ARG;
    if (in->m > 0 && !w_obs) return CAKF_E_ARG;
    hipStream_t st = c->stream;
    const int n = c->n, m = in->m, imax = c->imax, bsp = c->bsp;
    // B = a ws_{k+1} (padded to np rows), Y = sigma_f2 K(X, X) B
    launch_sample_scale_pad(ws_next, ns, (float)c->cfg.ou_coeff, n, c->np, ns, c->sp_W, bsp, st);
    launch_block_product(c->cfg.kernel, c->cfg.dist, c->cfg.prec, c->Xs, n, c->Xp, n, c->np,
                         c->sp_W, bsp, ns, c->sp_Bth, c->sp_Btl, (float)c->cfg.signal_var,
                         c->sp_Y, bsp, st, block_product_splits(n, c->np, ns, c->bpart_elems),
                         c->bpart);
    // xs = x + Y - M (M^T B)
    if (xs_out != x) launch_copy_rows(x, ns, xs_out, ns, n, ns, st);
    launch_add_cols(c->sp_Y, bsp, n, ns, xs_out, ns, st);
    if (rank > 0) {
        BLAS_TRY(sgemm_rm(c->blas, true, false, rank, ns, n, 1.0f, factor, ld, c->sp_W, bsp, 0.0f,
                          c->sp_Q, bsp));
        BLAS_TRY(sgemm_rm(c->blas, false, false, n, ns, rank, -1.0f, factor, ld, c->sp_Q, bsp,
                          1.0f, xs_out, ns));
    }
    if (m > 0) {
        // Pm = Y - M^- (M^-^T B) in place; WR = W_obs W_obs^T Pm[idx]
        if (in->pred_rank > 0) {
            BLAS_TRY(sgemm_rm(c->blas, true, false, in->pred_rank, ns, n, 1.0f, in->pred_factor,
                              in->pred_ld, c->sp_W, bsp, 0.0f, c->sp_Q, bsp));
            BLAS_TRY(sgemm_rm(c->blas, false, false, n, ns, in->pred_rank, -1.0f,
                              in->pred_factor, in->pred_ld, c->sp_Q, bsp, 1.0f, c->sp_Y, bsp));
        }
        launch_gather_rows(c->sp_Y, bsp, in->idx, m, n, ns, c->sp_D, bsp, st);
        BLAS_TRY(sgemm_rm(c->blas, true, false, imax, ns, m, 1.0f, in->W_obs, imax, c->sp_D, bsp,
                          0.0f, c->sp_R, bsp));
        BLAS_TRY(sgemm_rm(c->blas, false, false, m, ns, imax, 1.0f, in->W_obs, imax, c->sp_R, bsp,
                          0.0f, c->sp_D2, bsp));
    }
    // ws = B + H^T (wobs - WR)
    launch_copy_rows(c->sp_W, bsp, ws_out, ns, n, ns, st);
    if (m > 0)
        launch_sample_scatter(in->idx, n, m, ns, w_obs, ns, c->sp_D2, bsp, ws_out, ns, st);
    return hipGetLastError() == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

extern "C" int cakf_step(cakf_ctx* c, const int32_t* idx, const float* y, int m,
                         const float* actions, const cakf_record* rec) {
    if (!c) return CAKF_E_ARG;
    int rc;
    {
        PhaseTimer t(c, CAKF_PHASE_PREDICT);
        rc = cakf_predict(c);
    }
    if (rc) return rc;
    {
        PhaseTimer t(c, CAKF_PHASE_UPDATE);
        rc = cakf_update(c, idx, y, m, actions, rec);
    }
    if (rc) return rc;
    PhaseTimer t(c, CAKF_PHASE_TRUNCATE);
    return cakf_truncate(c, nullptr);
}

extern "C" int cakf_profile_enable(cakf_ctx* c, int on) {
    if (!c) return CAKF_E_ARG;
    c->prof.mask = on & ((1 << CAKF_PHASES) - 1);
    if (!on) {
        prof_free(c);
        return CAKF_OK;
    }
    if (!c->prof.on) {
        for (int p = 0; p < CAKF_PHASES; ++p)
            for (int k = 0; k < 2; ++k) {
                c->prof.ev[p][k] = new (std::nothrow) hipEvent_t[Prof::CAP];
                if (!c->prof.ev[p][k]) return CAKF_E_NOMEM;
                for (int e = 0; e < Prof::CAP; ++e)
                    HIP_TRY(hipEventCreate(&c->prof.ev[p][k][e]));
            }
        c->prof.on = true;
    }
    for (int p = 0; p < CAKF_PHASES; ++p) c->prof.count[p] = c->prof.seen[p] = 0;
    return CAKF_OK;
}

extern "C" int cakf_profile_stride(cakf_ctx* c, int every) {
    if (!c || every < 1) return CAKF_E_ARG;
    c->prof.stride = every;
    return CAKF_OK;
}

extern "C" int cakf_profile_read(cakf_ctx* c, double* total_ms, int* launches) {
    if (!c || !total_ms || !launches) return CAKF_E_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int p = 0; p < CAKF_PHASES; ++p) {
        double acc = 0.0;
        const int n = c->prof.on ? c->prof.count[p] : 0;
        for (int e = 0; e < n; ++e) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, c->prof.ev[p][0][e], c->prof.ev[p][1][e]));
            acc += ms;
        }
        total_ms[p] = acc;
        launches[p] = n;
        if (c->prof.on) c->prof.count[p] = c->prof.seen[p] = 0;
    }
    return CAKF_OK;
}

extern "C" int cakf_profile_rates(double* lanes_per_s) {
    if (!lanes_per_s) return CAKF_E_ARG;
    return probe_rates(lanes_per_s) == hipSuccess ? CAKF_OK : CAKF_E_HIP;
}

extern "C" int cakf_marginal_var(cakf_ctx* c, const int32_t* rows, int count, float* out) {
    if (!c || !out || count < 0) return CAKF_E_ARG;
    if (!rows && count != c->n) return CAKF_E_ARG;
    if (count == 0) return CAKF_OK;
    launch_marginal_var(c->M[c->cur], c->n, c->ldM, c->rank, (float)c->cfg.signal_var, rows,
                        count, out, c->stream);
    return CAKF_OK;
}

extern "C" int cakf_loglik(cakf_ctx* c, double* value, int* steps) {
    if (!c || !value) return CAKF_E_ARG;
    Diag h;
    HIP_TRY(hipMemcpyAsync(&h, c->diag, sizeof(Diag), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *value = h.loglik;
    if (steps) *steps = h.steps;
    return CAKF_OK;
}

extern "C" int cakf_diagnostics(cakf_ctx* c, int* dropped, int* nonfinite, int* bad_index) {
    if (!c) return CAKF_E_ARG;
    Diag h;
    HIP_TRY(hipMemcpyAsync(&h, c->diag, sizeof(Diag), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (dropped) *dropped = h.dropped;
    if (nonfinite) *nonfinite = h.nonfinite;
    if (bad_index) *bad_index = h.bad_index;
    return CAKF_OK;
}
