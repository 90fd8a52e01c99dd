// Host-side launchers of the libcakf kernels (one translation unit per kernel group).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "obs_types.h"

namespace cakf {

// Shape of the next_action launch: factor columns per lane (ldmo <= 64 CPL), action columns
// per lane (imax <= 64 LPL) and rows per wave (fewer when the rows' registers are large).
constexpr int next_action_cpl(int ldmo) { return ldmo <= 256 ? 4 : ldmo <= 512 ? 8 : 16; }
constexpr int next_action_lpl(int imax) { return imax <= 64 ? 1 : imax <= 128 ? 2 : 4; }
constexpr int next_action_rows_per_wave(int cpl, int lpl) { return (cpl > 8 || lpl > 2) ? 4 : 8; }
constexpr int next_action_blocks(int m, int cpl, int lpl) {
    return (m + 4 * next_action_rows_per_wave(cpl, lpl) - 1) /
           (4 * next_action_rows_per_wave(cpl, lpl));
}

// Direct mode of the Cholesky step (block-residual rounds): the Gram columns of the
// actions come ready from a round's product G (ld columns; row l = action l): columns
// uc + g, sc + g, vc + g hold s_l^T u_g, s_l^T s_g, s_l^T v_g of the round's action g,
// column rc holds s_l^T r0.
struct TailDirect {
    const double* G = nullptr;
    int ld = 0, uc = 0, sc = 0, vc = 0, rc = 0;
};

// ---- misc.hip
void launch_prescale(const float* X, int n, int dim, float c, int dist, float4* Xs,
                     hipStream_t st);
void launch_scale_state(float* mean, float* M, int n, int ld, int rank, float a, hipStream_t st);
void launch_mean_add(float* mean, const float* M, int n, int ld, int col, hipStream_t st);
void launch_predict_pairs(float* mean, float* M, int n, int ld, int rank, const float t[4],
                          hipStream_t st);
void launch_zero_cols(float* M, int ld, int rows, int cols, hipStream_t st);
void launch_fill_zero(float* p, size_t count, hipStream_t st);
void launch_marginal_var(const float* M, int n, int ld, int rank, float sigma_f2,
                         const int32_t* rows, int count, float* out, hipStream_t st);
void launch_copy_rows(const float* src, int lds, float* dst, int ldd, int rows, int cols,
                      hipStream_t st);

// ---- obs_loop.hip (launch_sym_tiles: sym_tiles.hip)
void launch_gather(const float4* Xs, int n, const float* mean, const float* M, int ldM,
                   const int32_t* idx, const float* y, const float* given, int cg,
                   const ObsDims& d, float4* Xo, float* r0, float* Mo, float* S, float* U,
                   LoopState* ls, hipStream_t st);
void launch_colsum_partial(const float* A, int lda, int rows, int cols, const float* x,
                           int ldx, float* partial, int ldp, hipStream_t st, int* nblk_out);
void launch_colsum_final(const float* partial, int ldp, int nblk, int cols, float* out,
                         int ldo, hipStream_t st);
// Offsets in the buffer of triangular products of an action's Cholesky step
// (tri_elems(imax) doubles): lrow and nrow (imax each), then the scalars l2 = |lrow|^2,
// la = lrow^T alpha and t_j^T t_j.
__host__ __device__ constexpr int tri_lrow(int imax) { return 0 * imax; }
__host__ __device__ constexpr int tri_nrow(int imax) { return 1 * imax; }
__host__ __device__ constexpr int tri_scal(int imax) { return 2 * imax; }
__host__ __device__ constexpr int tri_elems(int imax) { return 2 * imax + 3; }

// Inputs and outputs of the triangular products, taken by the last spare block of an
// action's sym_tiles launch: L^{-1} and its transpose (FP64, row-major, ld imax), alpha,
// the spare blocks' shares of T^T t_j (ceil(ldmo / 32) x imax doubles), the output
// buffer and the launch's arrival counter (one word, zero between launches; every launch
// leaves it at zero).
struct TriArgs {
    double* ttpart = nullptr;
    const double* Linv = nullptr;
    const double* LinvT = nullptr;
    const double* alpha = nullptr;
    double* tri = nullptr;
    unsigned* ctr = nullptr;
    double noise_var = 0.0;
};

// The O(j) rest of the Cholesky step of action j (obs_loop.hip): form_u's per-block sums
// of s_j^T u_j, the triangular products, the column products of s_j, beta after action
// j - 1 (beta_in) and the buffer for beta after action j (beta_out, another buffer), the
// rows it extends, the Gram matrix S^T S it fills (row j: s_l^T s_j, l <= j; its log
// determinant is taken once the loop ends), and the loop's tolerances.
struct TailArgs {
    const double* fupart = nullptr;
    int nfu = 0;
    int imax = 0;
    const double* tri = nullptr;
    const double* colvec = nullptr;
    const double* beta_in = nullptr;
    double* beta_out = nullptr;
    double* Linv = nullptr;
    double* LinvT = nullptr;
    double* L = nullptr;
    double* alpha = nullptr;
    double* SS = nullptr;
    double noise_var = 0.0, resid_tol = 0.0, pivot_tol = 0.0;
};

// The action-loop matvec of action j (sym_tiles.hip).  mfma_dist: Euclidean Matern-3/2
// and -5/2 take the squared distances from FP32 MFMA (dot-product form); otherwise every
// entry uses the difference form on the VALU.
void launch_sym_tiles(int nu2, int dist, bool mfma_dist, const float4* Xo, const float* S,
                      const ObsDims& d, int j, float* part, const float* mpart, int nmpart,
                      float* T, const double* cpart, int ncpart, int gs, double* colvec,
                      const LoopState* ls, const TriArgs& ta, hipStream_t st,
                      hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// u_j = sum of the tile sums into U[:, j], and per-block sums of s_j^T u_j
void launch_form_u(const float* part, const float* S, float* U, const ObsDims& d, int j,
                   double sigma_f2, double* fupart, const LoopState* ls, hipStream_t st,
                   int* nblk_out);
// the step of the last action (no next action follows), the final beta into beta_final
// (beta_odd: the buffer of the odd actions), and the log determinant of S^T S over the
// kept actions with the log-likelihood term (work: imax x imax doubles)
void launch_tail_final(const TailArgs& ta, int j, const double* beta_odd, double* beta_final,
                       double* work, LoopState* ls, hipStream_t st);
// The Cholesky steps of a block-policy round (direct mode, td.G != nullptr): nj actions
// from jfirst on.
void launch_tail(const ObsDims& d, int jfirst, double noise_var, double resid_tol,
                 double pivot_tol, double* Linv, double* LinvT, double* L, double* LSinv,
                 double* LSinvT, double* alpha, double* beta, LoopState* ls, hipStream_t st,
                 const TailDirect& td, int nj);
void launch_block_residual(const float* U, const float* V, float* S, const float* r0,
                           const double* beta, float noise_var, const ObsDims& d, int j0, int bt,
                           const LoopState* ls, hipStream_t st);
// skinny products of a block-policy round (partial buffer: round_products_elems)
size_t round_products_elems(int m, int P, int Q);
// G (P x Q, ld ldg, FP64) = A^T B over m rows, A (m x P, ld lda) and B (m x Q, ld ldb)
// row-major FP64: slab partial products (part: atb64_part_elems doubles) summed in a fixed
// order.
size_t atb64_part_elems(int m, int P, int Q);
void launch_atb64(const double* A, int lda, const double* B, int ldb, int m, int P, int Q,
                  double* part, double* G, int ldg, hipStream_t st);
void launch_round_gram(const float* U, const float* V, const float* S, const float* r0,
                       const ObsDims& d, int j0, int bt, double* part, double* G, int ldg,
                       hipStream_t st);
void launch_round_mot(const float* Mo, const float* S, const ObsDims& d, int j0, int bt,
                      float* part, float* T, hipStream_t st);
// resid: the CG residual is the action (else the action is read from S); mopart: also form
// the per-block partial sums of Mo^T s_jt (always with resid), finished by the next
// sym_tiles launch into column jt of T
// ta: the Cholesky step of action jt - 1 to finish first (required with resid)
void launch_next_action(int resid, int mopart, const float* U, const float* Mo,
                        const float* r0, float* S, float* V, const float* T, float noise_var,
                        const ObsDims& d, int jt, float* mpart, double* cpart, int gs,
                        LoopState* ls, const TailArgs* ta, hipStream_t st, int* nblk_out);
void launch_build_block(const float* S, const double* LinvT, const double* beta,
                        const ObsDims& d, float* B, int ldb, int bp, float* rec_W,
                        float* rec_w, float* rec_S, const LoopState* ls, hipStream_t st);
void launch_finish_record(const LoopState* ls, const double* L, const double* Linv, int imax,
                          double* rec_chol, double* rec_chol_inv, double* rec_loglik, int* rec_n,
                          hipStream_t st);

// ---- block_product.hip
// fp32_col >= 0 (BF16 modes): that column is also summed in FP32 from the FP32 kernel
// entries (chunk sums in FP64) and replaces the column's MFMA result; the FP32 mode sums
// every column that way.
void launch_block_product(int nu2, int dist, int prec, const float4* Xs, int n,
                          const float4* Xo, int m, int mp, const float* B, int ldb, int bcols,
                          __bf16* Bth, __bf16* Btl, float sigma_f2, float* out, int ldo,
                          hipStream_t st, int nsplit = 1, float* part = nullptr,
                          int fp32_col = -1);
// number of observation-axis splits for a block product of n rows (see launch_block_product)
int block_product_splits(int n, int mp, int bcols, size_t part_elems);

// ---- sampler.hip
void launch_sample_predict(const float* x, const float* q, float a, int n, int ns, int ld,
                           float* out, hipStream_t st);
void launch_sample_innov(const float* y, const int32_t* idx, const float* x, int ldx,
                         const float* e, int lde, float sigma, int n, int m, int ns, float* d,
                         int ldd, hipStream_t st);
void launch_sample_solve(const double* Linv, int imax, const float* r, int ns, int ld, float* z,
                         hipStream_t st);
void launch_add_cols(const float* Y, int ldy, int n, int ns, float* out, int ldo,
                     hipStream_t st);
void launch_sample_scale_pad(const float* in, int ldi, float a, int n, int rows, int ns,
                             float* out, int ld, hipStream_t st);
void launch_sample_copy_pad(const float* in, int ldi, int n, int rows, int ns, float* out,
                            int ld, hipStream_t st);
void launch_sample_scatter(const int32_t* idx, int n, int m, int ns, const float* v, int ldv,
                           const float* WR, int ldr, float* out, int ldo, hipStream_t st);
void launch_gather_points(const float4* Xs, int n, const int32_t* idx, int m, int mp,
                          float4* Xo, hipStream_t st);

// ---- truncate.hip
// orth > 0 with lam: the leading orth x orth block of the Gram is diag(scale * lam) (known
// orthogonal columns); its full 64 x 64 tiles are not computed
void launch_gram64(const float* M, int n, int ldM, int K, double* G, double* work,
                   size_t work_elems, hipStream_t st, int orth = 0,
                   const double* lam = nullptr, double scale = 1.0);
// lam[c] (c < r) = src[K - 1 - c] if ascending, else src[c]
void launch_store_lam(const double* src, int K, int r, int ascending, double* lam,
                      hipStream_t st);
void launch_pick_rotation(const double* E, int K, int r, float* Vr, double* rot_out,
                          hipStream_t st);

// ---- smooth.hip
void launch_smooth_pack(const float* ws, const float* Ws, int ldw, int n, int np, int rs,
                        float a, float* Bs, int ldb, hipStream_t st);
void launch_smooth_out(const float* mean, const float* M, int ldm, int rank, float g,
                       const float* Z, int ldz, int b, int n, float sigma_f2, float* mean_out,
                       float* factor_out, int ldo, float* var_out, hipStream_t st);
void launch_gather_rows(const float* A, int lda, const int32_t* idx, int m, int n, int cols,
                        float* out, int ldo, hipStream_t st);
void launch_smooth_messages(const float* Bs, int ldb, int n, const int32_t* idx, int m, int i,
                            int rs, const float* w_obs, const float* W_obs, int imax,
                            const float* WR, int ldr, float* ws, float* Wc, int ldw,
                            hipStream_t st);
void launch_pad_points(const float4* Xs, int n, int np, float4* Xp, hipStream_t st);

// ---- eig.hip
constexpr int TD_MAXK = 1280;       // largest K of the one-launch tridiagonalisation
int tridiag_max_k();
int tridiag_workgroups(int K);
hipError_t launch_tridiag(const double* G, int K, double* V, double* tau, double* d, double* e,
                          double* pbuf, double* rowbuf, unsigned* ctr, int* abort_flag,
                          hipStream_t st);
// V_r = Q Z_r: element (k, c) of Z_r (the eigenvector of the c-th largest eigenvalue of the
// tridiagonal) at Z[k * zrs + c * zcs]
void launch_backtransform(const double* Z, long long zrs, long long zcs, const double* Vh,
                          const double* tau, int K, int r, float* Vr, double* rot,
                          hipStream_t st);
// the r largest eigenpairs of the symmetric tridiagonal (d, e) of order
// K <= tri_eigen_max_k(): Zr (row-major K x r, descending eigenvalues), orthogonal up to
// eps ||T|| / (absolute eigenvalue gap); work: tri_eigen_work_elems(K, r) doubles
int tri_eigen_work_elems(int K, int r);
int tri_eigen_max_k();
void launch_tri_eigen(const double* d, const double* e, int K, int r, double* work, double* Zr,
                      hipStream_t st);
// steps of the symmetric orthogonalisation Z X, X = I - E/2 + (3/8) E^2, E = Z^T Z - I
// (r x r, FP64): mode 0 turns Z^T Z into E in place, mode 1 writes X over E2 = E E
void launch_lowdin(double* E, double* E2, int r, int mode, hipStream_t st);

// ---- probe.hip
// lane operations per second of v_exp_f32, v_sqrt_f32 and v_fma_f32 (out: 3 doubles)
hipError_t probe_rates(double* out);

// ---- adjoint.hip
// launch shape of k_adj_tiles: gx blocks of 32 q-points x gy slices of rps p-points
void adj_tiles_geometry(int np_, int mq, int* gx, int* gy, int* rps);
// b columns in launches of at most 160 (adj_tiles_launches(b) of them); *nblocks = the
// per-block partials written into spart in all; returns the slice count gy or < 0
constexpr int adj_tiles_launches(int b) { return (b + 159) / 160; }
int launch_adj_tiles(int nu2, int dist, bool bbar, const float4* Xp, int np_, const float* Yp,
                     int ldy, const float4* Xq, int mq, const float* Bq, int ldb, int b,
                     float* bpart, int ldbp, size_t slice_stride, double* spart,
                     int* nblocks, hipStream_t st);
void launch_adj_bbar_reduce(const float* bpart, size_t slice_stride, int ldbp, int ns, int m,
                            int mp, int b, float scale, float* out, int ldo, hipStream_t st);
void launch_adj_scalars(const double* spart, int nblk, double ck, double cd, double* grad,
                        int ik, int id, hipStream_t st);
void launch_adj_pack_ybar(const float* Mb, int ldM, int rank, int imax, const float* mb, int n,
                          float* Yb, int bp, hipStream_t st);
void launch_adj_obs_prep(const float4* Xs, int n, const int32_t* idx, const float* y, int m,
                         int mp, float a, const float* mprev, const float* Mprev, int ldprev,
                         int rank, const float* W_obs, const float* w_obs, const float* S,
                         int imax, int bp, int ldmo, float4* Xo, float* Mo, float* Bq,
                         double* W64, double* Sr64, hipStream_t st);
void launch_to_f64(const float* A, int lda, int rows, int cols, double* out, int ldo,
                   hipStream_t st);
void launch_to_f32(const double* A, size_t total, float* out, hipStream_t st);
void launch_to_f32_t(const double* A, int rows, int cols, float* out, hipStream_t st);
void launch_adj_small(int J, int imax, const double* G1, const double* G2, const double* L,
                      const double* Linv, double* X1, double* X2, float* Cc, double* grad,
                      int inoise, hipStream_t st);
void launch_adj_scatter(const int32_t* idx, int m, int n, const float* Mob, int ldmo, int rank,
                        const float* Zr, int ldz, int imax, float* Mb, int ldM, float* mb,
                        hipStream_t st);
int launch_adj_predict(float* mb, const float* mprev, float* Mb, int ldM, const float* Mprev,
                       int ldprev, int rank, int n, float a, double* part, hipStream_t st);
void launch_sum_into(const double* part, int nblk, double* grad, int i, hipStream_t st);

}  // namespace cakf
