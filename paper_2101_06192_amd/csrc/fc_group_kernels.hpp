// Host-side launch wrappers of the group forest closeness kernels (group.hip).  Every wrapper
// enqueues on `stream` and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fc {

// Group forest closeness (group.hip): dense N x N binary64 matrices,
// N = group_dim(n) (n rounded up to 256), row-major.
uint32_t group_dim(uint32_t n);
size_t group_scratch_doubles(uint32_t N);  // scratch of launch_group_invert
uint32_t group_chunks(uint32_t n);  // row chunks of the column sums
// A = alpha L + I on the first n rows and columns (weighted when w is not
// null), identity on the padding.
hipError_t launch_group_build(const int32_t *row_ptr, const int32_t *col_idx, const double *w,
                              uint32_t n, double alpha, double *A, hipStream_t stream);
// A <- A^{-1} in place (SPD; blocked Gauss-Jordan; scratch of
// group_scratch_doubles(N) doubles).
hipError_t launch_group_invert(double *A, uint32_t N, double *scratch, hipStream_t stream);
// diag[v] = A[v][v]; sel[0] = min diagonal bits, sel[1] = smallest id with it
// (sel preset to all ones by the caller).
hipError_t launch_group_first(const double *A, uint32_t n, uint32_t N, double *diag,
                              unsigned long long *sel, hipStream_t stream);
// Omega -> inverse of L* grounded at v0, in place (slot v0 becomes u*); c: n scratch.
hipError_t launch_group_reground(double *A, uint32_t n, uint32_t N, uint32_t v0, double *c,
                                 hipStream_t stream);
// *out = trace over the first n slots; *piv = A[v][v] when v < n.
hipError_t launch_group_trace(const double *A, uint32_t n, uint32_t N, uint32_t v, double *out,
                              double *piv, hipStream_t stream);
// Column sums of squares per row chunk into part (chunks x N); with v < n
// first the downdate by vertex v (pivot *piv; cv, rv: n scratch).
hipError_t launch_group_colsq(double *A, uint32_t n, uint32_t N, uint32_t v, double *cv, double *rv,
                              const double *piv, double *part, hipStream_t stream);
// One greedy step s >= 1 with no host round trip: the gains |M e_j|^2 / M_jj of
// the vertices not taken, per-block maxima and diagonal sums (bmax, bid, bdiag:
// blocks of 256 ids), then on the largest gain's smallest id v: taken[v] = 1,
// gout[s] = v, *piv = M[v][v], *vsel = v, the downdate and the next column
// sums.  With fout not null, fout[s - 1] = tr M as the step found it (f(S) of
// step s - 1; the last step's f(S) is left to launch_group_trace).  No
// candidate: gout[s] = -1, *bad = 1, the matrix as it was.
hipError_t launch_group_step(double *A, uint32_t n, uint32_t N, double *part, uint8_t *taken,
                             unsigned long long *bmax, uint32_t *bid, double *bdiag,
                             unsigned long long *vsel, double *cv, double *rv, double *piv,
                             int32_t *gout, double *fout, uint32_t s, uint32_t *bad,
                             hipStream_t stream);

}  // namespace fc
