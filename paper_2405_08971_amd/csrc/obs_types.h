// Types shared by the observation-space kernels and their host code.
#pragma once

namespace cakf {

constexpr int SYM_TILE = 128;       // side of the symmetric kernel tiles of the action loop

// Device-resident scalars of one update's action loop.
struct LoopState {
    int stop;          // set once the loop has stopped (budget, tolerance or breakdown)
    int i_eff;         // actions kept so far
    int dropped;       // actions dropped on breakdown since the last reset
    int nonfinite;     // non-finite pivots since the last reset
    double logdet_c;   // log det S^T Ghat S of the kept actions
    double logdet_s;   // log det S^T S of the kept actions
    double alpha2;     // ||L^{-1} S^T r0||^2
    double q00;        // ||s_0||^2 (CG: ||r0||^2)
    double loglik;     // projected log-likelihood term of the kept actions
    int bad_index;     // observation indices outside [0, n) seen by the gather
};

// Shapes shared by the observation-space kernels.
struct ObsDims {
    int m;        // observations
    int mp;       // m rounded up to SYM_TILE
    int imax;     // action budget; leading dimension of S, U, T and the FP64 triangles
    int rank;     // columns of the predictive factor
    int ldmo;     // leading dimension of Mo and T (max_rank rounded up to 8)
};

}  // namespace cakf
