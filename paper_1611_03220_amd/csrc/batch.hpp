// Batched solve: per-problem metadata and work items shared by host and device code.
#pragma once
#include "kernels.hpp"

namespace krr {

struct BatchMeta {
  int64_t off, n;          // packed row offset (multiple of ROW_PAD) and row count
  int m;                   // this problem's right-hand sides (<= packed width M)
  int nsplit;              // column splits of its kernel product
  double* part;            // its kernel-product partials [nsplit][rows_pad][M]
  int64_t part_stride;
  double lambda;           // ridge
  int red_begin, red_end;  // its reduction items
  int has_u;               // preconditioned
  const float* Ut;         // n x s (ldu)
  int64_t s, ldu;
  double inv_lp;           // 1 / lambda_p
  int pc_chunks;           // row chunks of the preconditioner's first pass
  int64_t pc_part_off;     // offset of its first-pass partials
  int64_t t_off;           // offset of its T = Ut^T r ([s][16])
  const double* ext_in;    // caller's Y (n x m, ld_in)
  int64_t ld_in;
  double* ext_out;         // caller's alpha (n x m, ld_out)
  int64_t ld_out;
};

struct RedItem { int inst; int64_t r0, r1; };             // packed row range of one problem
struct PCItem { int inst; int chunk; int64_t k0, i0, i1, part_off; };
struct ZItem { int inst; int64_t i0; };

struct BatchScalars {
  double *ynorm, *rnorm, *rho, *alpha, *beta;
  int *active, *broken, *col_iters, *count, *iter;
  int* live;  // per problem: 1 while any of its columns is active
  double* tol;  // per (problem, column) relative tolerance; >= 1 leaves the column inactive
};

// Kernels below take `live` (per problem, 1 while any of its columns is active) and skip the
// work of problems that have converged.
template <typename TA, typename TB>
hipError_t batch_dot(const TA* a, const TB* b, int M, const RedItem* items, int nitems,
                     const int* live, double* part, hipStream_t st);
hipError_t batch_init_scalars(const BatchMeta* meta, int count, int M, const double* part_yy,
                              const double* part_rz, BatchScalars& S, hipStream_t st);
hipError_t batch_alpha(const BatchMeta* meta, int count, int M, const double* part_pq,
                       BatchScalars& S, hipStream_t st);
hipError_t batch_conv(const BatchMeta* meta, int count, int M, const double* part_rr,
                      BatchScalars& S, hipStream_t st);
hipError_t batch_beta(const BatchMeta* meta, int count, int M, const double* part_rz,
                      const double* part_rr, BatchScalars& S, hipStream_t st);
hipError_t batch_finalize(const BatchMeta* meta, const int* row_inst, const int* live,
                          int64_t nrows, int M, const float* pf, double* q, hipStream_t st);
hipError_t batch_update_xr(const int* row_inst, int64_t nrows, int M, const double* alpha,
                           const float* pf, const double* q, double* x, double* r,
                           hipStream_t st);
hipError_t batch_update_p(const int* row_inst, int64_t nrows, int M, const double* beta,
                          const int* active, int init, const double* z, double* p, float* pf,
                          hipStream_t st);
hipError_t batch_split_v(const int* row_inst, const BatchMeta* meta, const int* live, int count,
                         int64_t nrows, int M, float* pf, const RedItem* items, int nitems,
                         float* colmax, _Float16* hi, _Float16* lo, float* vscale, bool packed,
                         hipStream_t st);
hipError_t batch_precond(const BatchMeta* meta, int count, const PCItem* pitems, int npitems,
                         const ZItem* zitems, int nzitems, int64_t smax, const int* live,
                         const double* r, int M, double* part, double* T, double* z,
                         hipStream_t st);
// mode: BATCH_PACK_IN (caller's Y -> packed), BATCH_UNPACK_SET / BATCH_UNPACK_ADD
// (packed -> caller's alpha, assigned or added)
enum { BATCH_UNPACK_SET = 0, BATCH_PACK_IN = 1, BATCH_UNPACK_ADD = 2 };
hipError_t batch_pack(const int* row_inst, const BatchMeta* meta, int64_t nrows, int M,
                      int mode, double* packed, hipStream_t st);

}  // namespace krr
