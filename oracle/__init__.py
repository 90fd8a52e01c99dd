"""Plain FP64 CPU oracle for the computation-aware Kalman filter and smoother.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call this
package: only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU library; both receive the same seeded inputs.

Modules
  matern  - half-integer Matern covariance functions and distances (App. D model).
  kalman  - textbook Kalman filter, RTS smoother and joint-Gaussian conditioning
            (Sec. 2.1, Thm. A.1, Thm. A.3), used to pin the computation-aware versions.
  cakf    - computation-aware Kalman filter: predict, iterative and batch update
            (Alg. 2 and the iterative Alg. in App. B), policies (Sec. 3.3, App. E),
            truncation (Sec. 3.2), per-step projected log-likelihood.
  caks    - computation-aware RTS smoother (Alg. 3).
  grad    - derivative of the projected log-likelihood with frozen actions and
            frozen truncation rotations (central differences in FP64).
"""
