// C ABI of libkrr: argument checks, workspace layout, and the PCG driver (Alg. 1).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/krr.h"
#include "kernels.hpp"

using namespace krr;

namespace {

thread_local char g_err[512] = "";

krr_status fail(krr_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define CHECK_HIP(...)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (__VA_ARGS__);                                                        \
    if (e_ != hipSuccess)                                                                 \
      return fail(KRR_E_HIP, "%s failed: %s (line %d)", #__VA_ARGS__, hipGetErrorString(e_), \
                  __LINE__);                                                              \
  } while (0)

#define CHECK_ST(expr)                     \
  do {                                     \
    krr_status s_ = (expr);                \
    if (s_ != KRR_OK) return s_;           \
  } while (0)

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<char*>(b)) {}
  template <typename T> T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

constexpr int NBLK = 256;  // blocks of the column-wise reductions

bool prec_ok(int32_t p) { return p == KRR_PREC_FP64 || p == KRR_PREC_F16X3 || p == KRR_PREC_BF16X3; }

int64_t kp_for(int64_t d) { return round_up(d + 2, K_STEP); }
// The F16X3 product uses MFMA accumulation (up to 32 columns of V per pass) for every d;
// the BF16X3 product keeps the VALU-accumulate kernel.
// (d + 3 <= 128: row operands in registers; larger d: both operands through LDS)
bool use_pv(int prec, int64_t d) { return prec == KRR_PREC_F16X3; }
int64_t kp_for(int prec, int64_t d) {
  return use_pv(prec, d) ? round_up(d + 2 + (PSHIFT > 0), K_STEP) : kp_for(d);
}
// FP64 point width: multiples of 8 up to 128 (FP64 MFMA kernel), else of 32 (VALU kernel)
// right-hand-side columns per pass of the MFMA-accumulate product: 32, or 160 for large d
// (where the distance work of a pass dominates its P V work: up to 160 columns share one
// distance pass)
int64_t pv_pass_width(int64_t Kp) { return Kp > 128 ? 160 : 32; }
// rows of the split V^T operand for a pass of mc columns: 16, 32, 64 or 160 (NCT = 1, 2, 4,
// 10)
int64_t pv_pass_rows(int64_t mc) { return mc > 64 ? 160 : mc > 32 ? 64 : round_up(mc, 16); }
int64_t dp_for(int64_t d) { return round_up(d, 8) <= 128 ? round_up(d, 8) : round_up(d, 32); }

// Split of the column sweep over blockIdx.y so that small row counts still fill the chip.
int choose_nsplit(int64_t n1, int64_t n2) {
  const int64_t rowblocks = ceil_div(n1, 128);
  const int64_t tiles = ceil_div(n2, 64);
  int64_t ns = ceil_div(2048, rowblocks);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, tiles / 4));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ns, 64));
}

// --------------------------------------------------------- kernel-product context
struct MatmatCtx {
  int prec = KRR_PREC_F16X3;
  bool pv = false;          // MFMA-accumulate kernel
  _Float16 *Vth = nullptr, *Vtl = nullptr;  // [mpad][rp2] split V^T (pv)
  float *colmax = nullptr, *vscale = nullptr;
  int64_t mpad = 0;
  int64_t n1 = 0, n2 = 0, d = 0, m = 0;
  int64_t rp1 = 0, rp2 = 0, Kp = 0, dp = 0;
  // Gaussian F16X3 products whose d + 2 crosses a 32-column step: the norm terms of the
  // exponent go to the epilogue (nrmA/nrmB, -q^2 c nu per row) and the operands are Kp_run =
  // round_up(d, 32) wide; Kp stays the augmented width (workspace and tuning key)
  float *nrmA = nullptr, *nrmB = nullptr;
  bool ne = false;
  int64_t Kp_run = 0;
  int nsplit = 1;
  int nsplit_max = 1;       // splits the partial buffer holds (tuned choices stay within it)
  int pass_w = 0;           // right-hand-side pass width (0: pv_pass_width)
  float* stats = nullptr;   // [0] max|x|, [1] max nu, [2] 1/q^2
  void *Ahi = nullptr, *Alo = nullptr, *Bhi = nullptr, *Blo = nullptr;
  double *nuA = nullptr, *nuB = nullptr;
  float *XAf = nullptr, *XBf = nullptr;  // FP32 coordinates of the large-d FP64 product
  int8_t *SA = nullptr, *SB = nullptr;    // int8 slices of the FP64 product (d <= 128)
  double *scA = nullptr, *scB = nullptr;  // their row scales
  double* part = nullptr;   // nsplit x rp1 x m
  int64_t part_stride = 0;
  // square large-d products: column-side accumulator of the symmetric kernel
  unsigned long long* fx = nullptr;  // [rp1][32]
  unsigned* fxflag = nullptr;        // [rp1]
  // square large-d FP64 products: two-word column-side accumulator of the symmetric kernel
  unsigned long long *fh = nullptr, *fl = nullptr;  // [rp1][16]
  unsigned* fflag = nullptr;                         // [rp1]
  unsigned long long* fvmax = nullptr;  // [16]
  bool square = false;
  double c2 = 0;            // log2(e) / (2 sigma^2)
  double sigma = 0;
  bool poly = false;        // polynomial kernel (gamma x^T z + c)^q instead of the Gaussian
  PolyF64 pk;               // its parameters
};

// square: both sides are the same points (the symmetric large-d kernel may be used);
// sym_buf: reserve its column-side accumulator (square, or a product whose sides may be the
// same points, sized before that is known)
void layout_matmat(Bump& b, MatmatCtx& c, int64_t n1, int64_t n2, int64_t d, int64_t m, int prec,
                   bool square, bool sym_buf) {
  c.prec = prec;
  c.square = square;
  c.n1 = n1; c.n2 = n2; c.d = d; c.m = m;
  c.rp1 = round_up(n1, ROW_PAD);
  c.rp2 = round_up(n2, ROW_PAD);
  c.nsplit = choose_nsplit(n1, n2);
  c.stats = b.take<float>(64);
  if (prec == KRR_PREC_FP64) {
    c.dp = dp_for(d);
    if (c.dp <= 128) {
      c.SA = b.take<int8_t>(c.rp1 * OZ_SLICES * oz_kp(d));
      c.scA = b.take<double>(c.rp1);
      if (!square) {
        c.SB = b.take<int8_t>(c.rp2 * OZ_SLICES * oz_kp(d));
        c.scB = b.take<double>(c.rp2);
      }
    } else {
      c.XAf = b.take<float>(c.rp1 * c.dp);
      if (!square) c.XBf = b.take<float>(c.rp2 * c.dp);
      if (sym_buf) {
        c.fh = b.take<unsigned long long>(c.rp1 * 16);
        c.fl = b.take<unsigned long long>(c.rp1 * 16);
        c.fflag = b.take<unsigned>(c.rp1);
        c.fvmax = b.take<unsigned long long>(16);
      }
    }
    c.nuA = b.take<double>(c.rp1);
    if (square) { c.XBf = c.XAf; c.SB = c.SA; c.scB = c.scA; c.nuB = c.nuA; }
    else c.nuB = b.take<double>(c.rp2);
  } else {
    c.pv = use_pv(prec, d);
    c.Kp = kp_for(prec, d);
    // the symmetric large-d kernel runs 256-row blocks: rows padded to 256
    if (c.pv && c.Kp > 128 && sym_buf) {
      c.rp1 = round_up(n1, 2 * ROW_PAD);
      c.rp2 = round_up(n2, 2 * ROW_PAD);
    }
    // large-d MFMA product on many row blocks: 8 column splits, launched in XCD groups
    if (c.pv && c.Kp > 128 && ceil_div(n1, 128) >= 64) c.nsplit = 8;
    if (c.pv) {
      // (a tuned pass width for large d is 32, 64 or 160, never above the default 160)
      c.mpad = pv_pass_rows(std::min<int64_t>(m, pv_pass_width(c.Kp)));
      c.Vth = b.take<_Float16>(c.mpad * c.rp2);
      c.Vtl = b.take<_Float16>(c.mpad * c.rp2);
      c.colmax = b.take<float>(m);
      c.vscale = b.take<float>(c.mpad);
    }
    if (c.pv && c.Kp > 128 && sym_buf) {
      c.fx = b.take<unsigned long long>(c.rp1 * 32);
      c.fxflag = b.take<unsigned>(c.rp1);
    }
    if (c.pv && c.Kp <= 128 && round_up(d, K_STEP) < c.Kp) {
      c.nrmA = b.take<float>(c.rp1);
      c.nrmB = b.take<float>(c.rp2);
    }
    c.Ahi = b.take<uint16_t>(c.rp1 * c.Kp);
    c.Alo = b.take<uint16_t>(c.rp1 * c.Kp);
    c.Bhi = b.take<uint16_t>(c.rp2 * c.Kp);
    c.Blo = b.take<uint16_t>(c.rp2 * c.Kp);
  }
  // the tuning table may pick fewer splits, or 8 where the rule picks fewer; the partial
  // buffer holds the larger of the two so the workspace size does not depend on the table
  c.nsplit_max = std::max(c.nsplit, 8);
  TuneChoice tc;
  if (tune_lookup(prec, 0, prec == KRR_PREC_FP64 ? c.dp : c.Kp, m, n1, &tc)) {
    if (tc.nsplit >= 1 && tc.nsplit <= c.nsplit_max) c.nsplit = tc.nsplit;
    if (tc.pass_width == 32 || tc.pass_width == 64 || tc.pass_width == 160)
      c.pass_w = tc.pass_width;
  }
  c.part_stride = c.rp1 * m;
  c.part = b.take<double>(c.nsplit_max * c.part_stride);
}

// Prepare both point sets for a kernel (X2 == nullptr: square product of X1).
hipError_t prepare_points(MatmatCtx& c, const float* X1, int64_t ldx1, const float* X2,
                          int64_t ldx2, const krr_kernel& k, hipStream_t st) {
  c.poly = k.kind == KRR_KERNEL_POLYNOMIAL;
  c.sigma = c.poly ? 1.0 : k.sigma;
  c.c2 = 1.4426950408889634 / (2.0 * c.sigma * c.sigma);
  c.pk.gamma = k.gamma;
  c.pk.coef0 = k.coef0;
  c.pk.deg = c.poly ? k.degree : 1;
  RowSpec rs;
  rs.poly = c.poly ? 1 : 0;
  rs.deg = c.pk.deg;
  rs.c2 = c.c2;
  rs.gamma = k.gamma;
  rs.coef0 = k.coef0;
  hipError_t e;
  if (c.prec == KRR_PREC_FP64) {
    if (c.XAf) {
      if ((e = prep_points_f64x(X1, c.n1, c.d, ldx1, c.rp1, c.dp, c.XAf, c.nuA, st))) return e;
      if (X2 && (e = prep_points_f64x(X2, c.n2, c.d, ldx2, c.rp2, c.dp, c.XBf, c.nuB, st))) return e;
      return hipSuccess;
    }
    if ((e = prep_points_i8(X1, c.n1, c.d, ldx1, c.rp1, c.SA, c.scA, c.nuA, st))) return e;
    if (X2 && (e = prep_points_i8(X2, c.n2, c.d, ldx2, c.rp2, c.SB, c.scB, c.nuB, st))) return e;
    return hipSuccess;
  }
  if ((e = fill_f32(c.stats, 4, 0.0f, st))) return e;
  if ((e = point_stats(X1, c.n1, c.d, ldx1, c.stats, st))) return e;
  if (X2 && (e = point_stats(X2, c.n2, c.d, ldx2, c.stats, st))) return e;
  const float* Xb = X2 ? X2 : X1;
  const int64_t ldb = X2 ? ldx2 : ldx1;
  const int ps = c.pv ? PSHIFT : 0;
  c.ne = c.nrmA && !c.poly && ps == 0;
  c.Kp_run = c.ne ? round_up(c.d, K_STEP) : c.Kp;
  if (c.prec == KRR_PREC_F16X3) {
    if ((e = prep_points<_Float16>(X1, c.n1, c.d, ldx1, c.rp1, c.Kp_run, rs, c.stats, 0, ps,
                                   (_Float16*)c.Ahi, (_Float16*)c.Alo, c.stats + 2, st,
                                   c.ne ? c.nrmA : nullptr)))
      return e;
    return prep_points<_Float16>(Xb, c.n2, c.d, ldb, c.rp2, c.Kp_run, rs, c.stats, 1, ps,
                                 (_Float16*)c.Bhi, (_Float16*)c.Blo, nullptr, st,
                                 c.ne ? c.nrmB : nullptr);
  }
  if (c.poly) return hipErrorInvalidValue;  // BF16X3 products are Gaussian only
  if ((e = prep_points<__bf16>(X1, c.n1, c.d, ldx1, c.rp1, c.Kp, rs, c.stats, 0, 0,
                               (__bf16*)c.Ahi, (__bf16*)c.Alo, c.stats + 2, st)))
    return e;
  return prep_points<__bf16>(Xb, c.n2, c.d, ldb, c.rp2, c.Kp, rs, c.stats, 1, 0, (__bf16*)c.Bhi,
                             (__bf16*)c.Blo, nullptr, st);
}
hipError_t prepare_points(MatmatCtx& c, const float* X1, int64_t ldx1, const float* X2,
                          int64_t ldx2, double sigma, hipStream_t st) {
  krr_kernel k{};
  k.kind = KRR_KERNEL_GAUSSIAN;
  k.sigma = sigma;
  return prepare_points(c, X1, ldx1, X2, ldx2, k, st);
}

// Partial sums of K V (or dK/dsigma V) into c.part. V is FP32 (mixed) or FP64 (FP64 path).
// On the MFMA-accumulate path Vf (n2 x ldv) is split in place: on return it holds exactly the
// vector the product used.
hipError_t run_matmat(const MatmatCtx& c, float* Vf, const double* V64, int64_t ldv, bool deriv,
                      hipStream_t st) {
  const double sig3 = c.sigma * c.sigma * c.sigma;
  if (c.prec == KRR_PREC_FP64) {
    F64Points A{c.nuA, c.n1, c.dp, c.XAf, c.SA, c.scA, c.d};
    F64Points B{c.nuB, c.n2, c.dp, c.XBf, c.SB, c.scB, c.d};
    const int epi = c.poly ? KV_POLY : deriv ? KV_DSIGMA : KV_GAUSS;
    const F64SymBuf sb{c.fh, c.fl, c.fflag, c.fvmax};
    return matmat_f64(A, B, V64, ldv, c.m, epi, 1.0 / (2.0 * c.sigma * c.sigma), 1.0 / sig3, c.pk,
                      c.part, c.m, c.part_stride, c.nsplit, st, c.fh && c.square ? &sb : nullptr);
  }
  const float dscale = (float)(1.0 / (c.c2 * sig3));  // dk/dsigma = k * (-log2 k) / (c2 sigma^3)
  if (c.prec == KRR_PREC_F16X3) {
    const bool ne = c.ne && c.Kp_run > 0;
    const int64_t kpr = ne ? c.Kp_run : c.Kp;
    MixedPoints<_Float16> A{(const _Float16*)c.Ahi, (const _Float16*)c.Alo, c.n1, kpr, c.stats + 2,
                            ne ? c.nrmA : nullptr};
    MixedPoints<_Float16> B{(const _Float16*)c.Bhi, (const _Float16*)c.Blo, c.n2, kpr, c.stats + 2,
                            ne ? c.nrmB : nullptr};
    if (c.pv) {
      const int64_t W = c.Kp > 128 && c.pass_w ? c.pass_w : pv_pass_width(c.Kp);
      for (int64_t c0 = 0; c0 < c.m; c0 += W) {
        const int64_t mc = std::min<int64_t>(W, c.m - c0);
        const int64_t mp = pv_pass_rows(mc);
        if (mp > c.mpad) return hipErrorInvalidValue;  // V^T buffers hold c.mpad rows
        const bool packed = mc <= 8;  // hi and lo parts share one 16-row operand
        hipError_t e = vec_split_t(Vf + c0, c.n2, mc, ldv, c.rp2, mp, c.colmax, PSHIFT, packed,
                                   c.Vth, c.Vtl, c.vscale, st);
        if (e != hipSuccess) return e;
        SplitRhs V{c.Vth, c.Vtl, c.vscale, c.rp2, mp, packed};
        const int epi = c.poly ? KV_POLY : deriv ? KV_DSIGMA : KV_GAUSS;
        const SymBuf sb{c.fx, c.fxflag, 32};
        e = matmat_f16pv(A, B, V, mc, epi, dscale, c.part + c0, c.m, c.part_stride, c.nsplit, st,
                         c.fx && c.square ? &sb : nullptr);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    if (c.poly) return hipErrorInvalidValue;
    return matmat_mixed<_Float16>(A, B, Vf, ldv, c.m, deriv, dscale, c.part, c.m, c.part_stride,
                                  c.nsplit, st);
  }
  if (c.poly) return hipErrorInvalidValue;
  MixedPoints<__bf16> A{(const __bf16*)c.Ahi, (const __bf16*)c.Alo, c.n1, c.Kp, c.stats + 2};
  MixedPoints<__bf16> B{(const __bf16*)c.Bhi, (const __bf16*)c.Blo, c.n2, c.Kp, c.stats + 2};
  return matmat_mixed<__bf16>(A, B, Vf, ldv, c.m, deriv, dscale, c.part, c.m, c.part_stride,
                              c.nsplit, st);
}

krr_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return fail(KRR_E_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(KRR_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(KRR_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return KRR_OK;
}

// ------------------------------------------------------------------ features
struct FeatLayout {
  float* stats;
  _Float16 *Xh, *Xl, *Wh, *Wl;
  int64_t dk, np, sp;
};
void layout_features(Bump& b, FeatLayout& L, int64_t n, int64_t d, int64_t s) {
  L.dk = round_up(d, 32);
  L.np = round_up(n, GEMM_TILE);
  L.sp = round_up(s, GEMM_TILE);
  L.stats = b.take<float>(64);
  L.Xh = b.take<_Float16>(L.np * L.dk);
  L.Xl = b.take<_Float16>(L.np * L.dk);
  L.Wh = b.take<_Float16>(L.sp * L.dk);
  L.Wl = b.take<_Float16>(L.sp * L.dk);
}

// ------------------------------------------------------- Gaussian projection (Alg. 2)
struct ProjLayout {
  float* stats;
  _Float16 *Ah, *Al, *Bh, *Bl;
  int64_t kp, np, sp;
};
void layout_project(Bump& b, ProjLayout& L, int64_t n, int64_t s2, int64_t s3) {
  L.kp = round_up(s2, 32);
  L.np = round_up(n, GEMM_TILE);
  L.sp = round_up(s3, GEMM_TILE);
  L.stats = b.take<float>(64);
  L.Ah = b.take<_Float16>(L.np * L.kp);
  L.Al = b.take<_Float16>(L.np * L.kp);
  L.Bh = b.take<_Float16>(L.sp * L.kp);
  L.Bl = b.take<_Float16>(L.sp * L.kp);
}

// ---------------------------------------------------------------- precond factor
krr_status gram_cholesky(const float* Z, int64_t n, int64_t s, int64_t ldz, double lambda_p,
                         struct FactorLayout& L, int64_t* info, const char* fn, hipStream_t st);
int gram_nsplit(int64_t s, int64_t n) {
  const int64_t t = ceil_div(s, GEMM_TILE);
  const int64_t tiles = t * (t + 1) / 2;
  int64_t ns = ceil_div(1024, tiles);  // enough blocks; every split adds s^2 FP64 partials
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, ceil_div(n, 2048)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ns, 32));
}
struct FactorLayout {
  float* stats;
  _Float16 *h1, *l1;     // Zt split (sp64 x nk), later Z split (np x sk)
  _Float16 *ch, *cl;     // Cinv split (sp64 x sk)
  double *part, *G, *Cinv, *tmp;
  int* info;
  int64_t nk, sk, np, sp64, s_pad;
  int nsplit;
};
// `own` receives what one problem's factor keeps from the Gram to the end (scales, pivot
// flag, G, C^{-1}, doubling scratch), `scratch` the operand splits and Gram partials.
void layout_factor_parts(Bump& scratch, Bump& own, FactorLayout& L, int64_t n, int64_t s) {
  L.nk = round_up(n, 32);
  L.sk = round_up(s, 32);
  L.np = round_up(n, GEMM_TILE);
  L.sp64 = round_up(s, GEMM_TILE);
  L.s_pad = round_up(s, 64);  // 64 x 64 factor blocks
  L.nsplit = gram_nsplit(s, n);
  L.stats = own.take<float>(64);
  L.info = own.take<int>(64);
  const int64_t big = std::max(L.sp64 * L.nk, L.np * L.sk);
  L.h1 = scratch.take<_Float16>(big);
  L.l1 = scratch.take<_Float16>(big);
  L.ch = scratch.take<_Float16>(L.sp64 * L.sk);
  L.cl = scratch.take<_Float16>(L.sp64 * L.sk);
  L.part = scratch.take<double>((int64_t)L.nsplit * s * s);
  L.G = own.take<double>(L.s_pad * L.s_pad);
  L.Cinv = own.take<double>(L.s_pad * L.s_pad);
  L.tmp = own.take<double>(L.s_pad * L.s_pad / 2);
}
void layout_factor(Bump& b, FactorLayout& L, int64_t n, int64_t s) { layout_factor_parts(b, b, L, n, s); }

// G = Z^T Z + lambda_p I (split MFMA Gram, FP64 sums) and its FP64 Cholesky factor in L.G
// (stride s_pad); KRR_E_NOT_SPD with *info = failing pivot + 1.
krr_status gram_cholesky(const float* Z, int64_t n, int64_t s, int64_t ldz, double lambda_p,
                         FactorLayout& L, int64_t* info, const char* fn, hipStream_t st) {
  CHECK_HIP(fill_f32(L.stats, 4, 0.0f, st));
  CHECK_HIP(fill_i32(L.info, 1, 0, st));
  // Gram G = Z^T Z: A = B = Z^T (s x n, contraction over points)
  CHECK_HIP(absmax<float>(Z, n, s, ldz, L.stats + 0, st));
  CHECK_HIP((split_operand<float, _Float16>(Z, n, s, ldz, L.stats + 0, 1, L.sp64, L.nk, L.h1, L.l1, st)));
  SplitOperand Zt{L.h1, L.l1, L.nk, L.stats + 0};
  CHECK_HIP(gemm_nt_f16x3(Zt, Zt, s, s, L.nk, L.nsplit, EPI_PART64, 1, 0, 1.0, L.part, s * s,
                          nullptr, s, nullptr, 0.0f, st));
  CHECK_HIP(gram_finalize(L.part, L.nsplit, s, s, s * s, lambda_p, L.s_pad, L.G, st));
  // Cholesky (FP64)
  CHECK_HIP(fill_f64(L.Cinv, L.s_pad * L.s_pad, 0.0, st));
  CHECK_HIP(cholesky_blocked(L.G, L.s_pad, L.Cinv, L.info, st));
  int hinfo = 0;
  CHECK_HIP(hipMemcpyAsync(&hinfo, L.info, sizeof(int), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  if (hinfo != 0) {
    if (info) *info = hinfo;
    return fail(KRR_E_NOT_SPD, "%s: Z^T Z + lambda_p I not positive definite at pivot %d", fn, hinfo);
  }
  return KRR_OK;
}

// G = Z^T Z + lambda_p I in L.G (as gram_cholesky), C^{-1} cleared and the pivot flag reset,
// without the factor itself
hipError_t gram_form_async(const float* Z, int64_t n, int64_t s, int64_t ldz, double lambda_p,
                           FactorLayout& L, hipStream_t st) {
  hipError_t e;
  if ((e = fill_f32(L.stats, 4, 0.0f, st))) return e;
  if ((e = fill_i32(L.info, 1, 0, st))) return e;
  if ((e = absmax<float>(Z, n, s, ldz, L.stats + 0, st))) return e;
  if ((e = split_operand<float, _Float16>(Z, n, s, ldz, L.stats + 0, 1, L.sp64, L.nk, L.h1, L.l1, st))) return e;
  SplitOperand Zt{L.h1, L.l1, L.nk, L.stats + 0};
  if ((e = gemm_nt_f16x3(Zt, Zt, s, s, L.nk, L.nsplit, EPI_PART64, 1, 0, 1.0, L.part, s * s,
                         nullptr, s, nullptr, 0.0f, st))) return e;
  if ((e = gram_finalize(L.part, L.nsplit, s, s, s * s, lambda_p, L.s_pad, L.G, st))) return e;
  return fill_f64(L.Cinv, L.s_pad * L.s_pad, 0.0, st);
}

// after the Cholesky factor in L.G and C^{-1} in L.Cinv: C (lower, s x s), Ut = Z C^{-T}
hipError_t factor_tail(FactorLayout& L, const float* Z, int64_t n, int64_t s, int64_t ldz,
                       double* C, float* Ut, int64_t ldu, hipStream_t st) {
  hipError_t e;
  if ((e = copy_lower(L.G, L.s_pad, s, C, st))) return e;
  // Ut = Z C^{-T}: A = Z (n x s), B = C^{-1} (rows j, contraction k), lower triangular
  if ((e = absmax<double>(L.Cinv, s, s, L.s_pad, L.stats + 1, st))) return e;
  if ((e = split_operand<float, _Float16>(Z, n, s, ldz, L.stats + 0, 0, L.np, L.sk, L.h1, L.l1, st))) return e;
  if ((e = split_operand<double, _Float16>(L.Cinv, s, s, L.s_pad, L.stats + 1, 0, L.sp64, L.sk, L.ch, L.cl, st))) return e;
  SplitOperand A{L.h1, L.l1, L.sk, L.stats + 0}, B{L.ch, L.cl, L.sk, L.stats + 1};
  return gemm_nt_f16x3(A, B, n, s, L.sk, 1, EPI_F32, 0, 1, 1.0, nullptr, 0, Ut, ldu, nullptr, 0.0f,
                       st);
}

// after the Cholesky factor in L.G: C^{-1} by doubling, then factor_tail
hipError_t factor_finish(FactorLayout& L, const float* Z, int64_t n, int64_t s, int64_t ldz,
                         double* C, float* Ut, int64_t ldu, hipStream_t st) {
  hipError_t e;
  if ((e = tri_inverse_doubling(L.G, L.s_pad, L.Cinv, L.tmp, st))) return e;
  return factor_tail(L, Z, n, s, ldz, C, Ut, ldu, st);
}

// ---------------------------------------------------------------------- PCG
struct PCGLayout {
  MatmatCtx mm;      // kernel product in the solve precision
  MatmatCtx mm64;    // FP64 product for the true residual / refinement
  float* pf;         // FP32 copy of p (mixed)
  double *p, *q, *r, *z, *ax, *delta, *rhs;
  double *part_yy, *part_rr, *part_pq, *part_rz, *pc_part, *T;
  double *ynorm, *rnorm, *rho, *alpha, *beta, *hist;
  int *active, *broken, *col_iters, *count;
  int nchunk;
};
int precond_nchunk(int64_t n, int64_t s) {
  const int64_t kb = ceil_div(std::max<int64_t>(s, 1), 512);  // feature columns per block
  int64_t nc = ceil_div(1024, kb);
  nc = std::min<int64_t>(nc, std::max<int64_t>(1, ceil_div(n, 256)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(nc, 512));
}
void layout_pcg(Bump& b, PCGLayout& L, int64_t n, int64_t d, int64_t s, int64_t m, int prec) {
  layout_matmat(b, L.mm, n, n, d, m, prec, true, true);
  if (prec != KRR_PREC_FP64) layout_matmat(b, L.mm64, n, n, d, m, KRR_PREC_FP64, true, true);
  const int64_t nm = n * m;
  L.pf = b.take<float>(round_up(n, ROW_PAD) * m);
  L.p = b.take<double>(nm);
  L.q = b.take<double>(nm);
  L.r = b.take<double>(nm);
  L.z = b.take<double>(nm);
  L.ax = b.take<double>(nm);
  L.delta = b.take<double>(nm);
  L.rhs = b.take<double>(nm);
  L.part_yy = b.take<double>(NBLK * m);
  L.part_rr = b.take<double>(NBLK * m);
  L.part_pq = b.take<double>(NBLK * m);
  L.part_rz = b.take<double>(NBLK * m);
  L.nchunk = precond_nchunk(n, s);
  L.pc_part = b.take<double>((int64_t)L.nchunk * std::max<int64_t>(s, 1) * m);
  L.T = b.take<double>(std::max<int64_t>(s, 1) * m);
  L.ynorm = b.take<double>(m);
  L.rnorm = b.take<double>(m);
  L.rho = b.take<double>(m);
  L.alpha = b.take<double>(m);
  L.beta = b.take<double>(m);
  L.hist = b.take<double>(2);
  L.active = b.take<int>(m);
  L.broken = b.take<int>(m);
  L.col_iters = b.take<int>(m);
  L.count = b.take<int>(2);
}

struct GradLayout {
  MatmatCtx mm;
  float* af;   // FP32 copy of alpha for the mixed product
  double* w;
  double* part;
};
struct ApplyLayout {
  double *part, *T, *r, *z;
  int nchunk;
};
void layout_apply(Bump& b, ApplyLayout& L, int64_t n, int64_t s, int64_t m) {
  L.nchunk = precond_nchunk(n, s);
  L.part = b.take<double>((int64_t)L.nchunk * std::max<int64_t>(s, 1) * m);
  L.T = b.take<double>(std::max<int64_t>(s, 1) * m);
  L.r = b.take<double>(n * m);  // contiguous copies when the caller's are strided
  L.z = b.take<double>(n * m);
}

// <G, (dK(X1, X2)/dsigma) V>: cross product partials, FP32 V copy, the product, partial dots
struct InnerLayout {
  MatmatCtx mm;
  float* vf;
  double* w;
  double* part;
};
void layout_inner(Bump& b, InnerLayout& L, int64_t n1, int64_t n2, int64_t d, int64_t m, int prec) {
  layout_matmat(b, L.mm, n1, n2, d, m, prec, false, false);
  L.vf = prec != KRR_PREC_FP64 ? b.take<float>(round_up(n2, ROW_PAD) * m) : nullptr;
  L.w = b.take<double>(n1 * m);
  L.part = b.take<double>(NBLK * m);
}

// The Thm. 4 test of a candidate sketch Z (n x s): factor of Z^T Z + jitter, Jacobi
// eigen-decomposition, the orthonormal basis U_k of range(P) (n x s FP32 buffer), the kernel
// product of one vector, power-iteration vectors and reduction scratch.
struct TestLayout {
  FactorLayout F;
  MatmatCtx mm;
  double *Zd, *A, *Vt, *ev, *scale, *v, *w, *t, *x, *y, *part, *gpart, *T, *pc_part;
  float *Bk, *Uk, *vf;
  int* idx;
  unsigned long long* off;
  int nchunk;
};
void layout_test(Bump& b, TestLayout& L, int64_t n, int64_t d, int64_t s, int prec) {
  layout_factor(b, L.F, n, s);
  layout_matmat(b, L.mm, n, n, d, 1, prec, true, true);
  L.Zd = b.take<double>(n * s);
  L.A = b.take<double>(s * s);
  L.Vt = b.take<double>(s * s);
  L.ev = b.take<double>(s);
  L.scale = b.take<double>(s);
  L.idx = b.take<int>(s);
  L.off = b.take<unsigned long long>(1);
  L.Bk = b.take<float>(s * s);
  L.Uk = b.take<float>(n * s);
  L.vf = b.take<float>(round_up(n, ROW_PAD));
  L.v = b.take<double>(n);
  L.w = b.take<double>(n);
  L.t = b.take<double>(n);
  L.x = b.take<double>(s);
  L.y = b.take<double>(s);
  L.part = b.take<double>(NBLK * 2);
  L.gpart = b.take<double>(GEMV_PARTS_MAX * s);
  L.nchunk = precond_nchunk(n, s);
  L.pc_part = b.take<double>((int64_t)L.nchunk * s);
  L.T = b.take<double>(s);
}

// autotuning: the product, synthetic right-hand sides and their FP32 copy
struct TuneLayout {
  MatmatCtx mm;
  double *V, *out;
  float* Vf;
};
void layout_tune(Bump& b, TuneLayout& L, int64_t n, int64_t d, int64_t m, int prec) {
  layout_matmat(b, L.mm, n, n, d, m, prec, true, true);
  L.V = b.take<double>(n * m);
  L.out = b.take<double>(n * m);
  L.Vf = b.take<float>(round_up(n, ROW_PAD) * m);
}

void layout_grad(Bump& b, GradLayout& L, int64_t n, int64_t d, int64_t m, int prec) {
  layout_matmat(b, L.mm, n, n, d, m, prec, true, true);
  L.af = b.take<float>(round_up(n, ROW_PAD) * m);
  L.w = b.take<double>(n * m);
  L.part = b.take<double>(NBLK * m * 2);
}

}  // namespace

namespace krr {
krr_status report_error(krr_status code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace krr

// =================================================================== C ABI
extern "C" {

const char* krr_last_error(void) { return g_err; }
const char* krr_version(void) { return "libkrr 0.1 (gfx950)"; }

void krr_pcg_defaults(krr_pcg_opts* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->max_iter = 1000;
  o->prec = KRR_PREC_F16X3;
  o->use_precond = 1;
  o->check_every = 1;
  o->lambda_p = 0.0;
  o->true_residual = 1;
  o->refine = 0;
  o->warm_start = 0;
}

size_t krr_workspace_bytes(int32_t op, int64_t n1, int64_t n2, int64_t d, int64_t s, int64_t m,
                           int32_t prec) {
  if (n1 < 1 || d < 0 || s < 0 || m < 0) return 0;
  if (!prec_ok(prec)) prec = KRR_PREC_F16X3;
  Bump b(nullptr);
  switch (op) {
    case KRR_OP_FEATURES: { FeatLayout L; layout_features(b, L, n1, d, s); break; }
    case KRR_OP_PRECOND_FACTOR: { FactorLayout L; layout_factor(b, L, n1, s); break; }
    case KRR_OP_KERNEL_MATMAT: {
      MatmatCtx c;
      layout_matmat(b, c, n1, n2, d, m, prec, false, n1 == n2);
      if (prec != KRR_PREC_FP64) b.take<float>(round_up(n2, ROW_PAD) * m);
      break;
    }
    case KRR_OP_PCG_SOLVE: { PCGLayout L; layout_pcg(b, L, n1, d, s, m, prec); break; }
    case KRR_OP_GRAD: { GradLayout L; layout_grad(b, L, n1, d, m, prec); break; }
    case KRR_OP_PRECOND_APPLY: { ApplyLayout L; layout_apply(b, L, n1, s, m); break; }
    case KRR_OP_AUTOTUNE: { TuneLayout L; layout_tune(b, L, n1, d, m, prec); break; }
    case KRR_OP_ADAPTIVE_FEATURES: {
      if (s < 1) return 0;
      TestLayout L;
      layout_test(b, L, n1, d, s, prec);
      FeatLayout F;
      Bump fb(nullptr);
      layout_features(fb, F, n1, d, s);
      return std::max(b.off, fb.off) + 256;
    }
    case KRR_OP_PRECOND_TEST: {
      if (s < 1) return 0;
      TestLayout L;
      layout_test(b, L, n1, d, s, prec);
      break;
    }
    case KRR_OP_GAUSSIAN_PROJECT: {
      if (s < 1) return 0;
      ProjLayout L;
      layout_project(b, L, n1, d, s);
      break;
    }
    case KRR_OP_DSIGMA_INNER: {
      if (n2 < 1) return 0;
      InnerLayout L;
      layout_inner(b, L, n1, n2, d, m, prec);
      break;
    }
    default: return 0;
  }
  return b.off + 256;
}

// ------------------------------------------------------------------ features
namespace {
// Random Fourier features from the first s columns of W (d x ldw) and entries of b.
krr_status features_impl(const char* fn, const float* X, int64_t n, int64_t d, int64_t ldx,
                         const float* W, int64_t ldw, const float* b, int64_t s, float* Z,
                         int64_t ldz, void* ws, size_t ws_bytes, hipStream_t st);
}  // namespace

krr_status krr_features(const float* X, int64_t n, int64_t d, int64_t ldx, const float* W,
                        const float* b, int64_t s, float* Z, int64_t ldz, void* ws,
                        size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !W || !b || !Z) return fail(KRR_E_ARG, "krr_features: null pointer");
  if (n < 1 || d < 1 || s < 1 || ldx < d || ldz < s)
    return fail(KRR_E_ARG, "krr_features: bad sizes n=%lld d=%lld s=%lld", (long long)n,
                (long long)d, (long long)s);
  return features_impl("krr_features", X, n, d, ldx, W, s, b, s, Z, ldz, ws, ws_bytes,
                       (hipStream_t)stream);
}

namespace {
krr_status features_impl(const char* fn, const float* X, int64_t n, int64_t d, int64_t ldx,
                         const float* W, int64_t ldw, const float* b, int64_t s, float* Z,
                         int64_t ldz, void* ws, size_t ws_bytes, hipStream_t st) {
  Bump probe(nullptr);
  FeatLayout L;
  layout_features(probe, L, n, d, s);
  CHECK_ST(check_ws(ws, ws_bytes, probe.off + 256));
  (void)fn;
  Bump bb(ws);
  layout_features(bb, L, n, d, s);
  CHECK_HIP(fill_f32(L.stats, 4, 0.0f, st));
  CHECK_HIP(absmax<float>(X, n, d, ldx, L.stats + 0, st));
  CHECK_HIP(absmax<float>(W, d, s, ldw, L.stats + 1, st));
  CHECK_HIP((split_operand<float, _Float16>(X, n, d, ldx, L.stats + 0, 0, L.np, L.dk, L.Xh, L.Xl, st)));
  // W is d x s; its transpose (s x d, contraction index contiguous) is the B operand
  CHECK_HIP((split_operand<float, _Float16>(W, d, s, ldw, L.stats + 1, 1, L.sp, L.dk, L.Wh, L.Wl, st)));
  SplitOperand A{L.Xh, L.Xl, L.dk, L.stats + 0}, B{L.Wh, L.Wl, L.dk, L.stats + 1};
  CHECK_HIP(gemm_nt_f16x3(A, B, n, s, L.dk, 1, EPI_COS, 0, 0, 1.0, nullptr, 0, Z, ldz, b,
                          (float)std::sqrt(2.0 / (double)s), st));
  return KRR_OK;
}
}  // namespace

// ---------------------------------------------------------------- precond factor
krr_status krr_precond_factor(const float* Z, int64_t n, int64_t s, int64_t ldz, double lambda_p,
                              double* C, float* Ut, int64_t ldu, void* ws, size_t ws_bytes,
                              int64_t* info, void* stream) {
  g_err[0] = 0;
  if (!Z || !C || !Ut || !info) return fail(KRR_E_ARG, "krr_precond_factor: null pointer");
  *info = 0;
  if (n < 2 || s < 1 || s >= n || ldz < s || ldu < s)
    return fail(KRR_E_ARG, "krr_precond_factor: need 1 <= s < n and ld >= s (n=%lld s=%lld)",
                (long long)n, (long long)s);
  if (!(lambda_p > 0.0) || !std::isfinite(lambda_p))
    return fail(KRR_E_ARG, "krr_precond_factor: lambda_p must be > 0");
  Bump probe(nullptr);
  FactorLayout L;
  layout_factor(probe, L, n, s);
  CHECK_ST(check_ws(ws, ws_bytes, probe.off + 256));
  Bump bb(ws);
  layout_factor(bb, L, n, s);
  hipStream_t st = (hipStream_t)stream;
  CHECK_ST(gram_cholesky(Z, n, s, ldz, lambda_p, L, info, "krr_precond_factor", st));
  CHECK_HIP(factor_finish(L, Z, n, s, ldz, C, Ut, ldu, st));
  CHECK_HIP(hipStreamSynchronize(st));
  return KRR_OK;
}

// ------------------------------------------------ set-up of many problems on several streams
namespace {
// Per problem: its stream slot (the features, or the factor's operand splits and Gram
// partials) and what it keeps from its Gram to the end of the set-up (G, C^{-1}, scratch).
void setup_sizes(const krr_setup_problem& p, size_t& slot, size_t& own) {
  Bump f(nullptr), g(nullptr), o(nullptr);
  FeatLayout FL;
  layout_features(f, FL, p.n, p.d, p.s);
  FactorLayout L;
  layout_factor_parts(g, o, L, p.n, p.s);
  slot = (size_t)round_up((int64_t)std::max(f.off, g.off), 256) + 256;
  own = (size_t)round_up((int64_t)o.off, 256) + 256;
}

// The FP64 factors of all problems advance together: one launch per step covers every
// problem that still has it. GEMM lists: the trailing update after each 64-column block,
// then per doubling level the T = B A^{-1} products and the X = -D^{-1} T products (the
// pairs of tri_inverse_doubling, each pair one product, every problem's T in its own tmp).
struct GroupLaunch {
  int64_t off = 0, count = 0, max_m = 0, max_n = 0;
};
struct GroupedFactorPlan {
  std::vector<DgemmProblem> probs;
  std::vector<GroupLaunch> trail;   // column block k0 = 64 t
  std::vector<GroupLaunch> levels;  // T then X for b = 64, 128, ...
  int64_t max_s_pad = 0;
};
void add_problem(GroupLaunch& g, std::vector<DgemmProblem>& v, const DgemmProblem& p) {
  v.push_back(p);
  ++g.count;
  g.max_m = std::max(g.max_m, p.M);
  g.max_n = std::max(g.max_n, p.N);
}
void plan_grouped_factor(const std::vector<FactorLayout>& Ls, GroupedFactorPlan& P) {
  P = GroupedFactorPlan{};
  for (const FactorLayout& L : Ls) P.max_s_pad = std::max(P.max_s_pad, L.s_pad);
  for (int64_t k0 = 0; k0 < P.max_s_pad; k0 += 64) {
    GroupLaunch g;
    g.off = (int64_t)P.probs.size();
    for (const FactorLayout& L : Ls) {
      const int64_t sp = L.s_pad, rest = sp - k0 - 64;
      if (rest <= 0) continue;
      double* panel = L.G + (k0 + 64) * sp + k0;
      add_problem(g, P.probs, DgemmProblem{panel, panel, panel + 64, sp, 1, 1, sp, sp, rest, rest,
                                           64, -1.0, 1.0, 1});
    }
    P.trail.push_back(g);
  }
  for (int64_t b = 64; b < P.max_s_pad; b *= 2) {
    GroupLaunch t, x;
    t.off = (int64_t)P.probs.size();
    for (const FactorLayout& L : Ls) {
      const int64_t sp = L.s_pad;
      if (b >= sp) continue;
      const int64_t full = sp / (2 * b);
      for (int64_t q = 0; q <= full; ++q) {
        const int64_t o1 = 2 * b * q, o2 = o1 + b, rows = std::min(b, sp - o2);
        if (rows <= 0) break;
        add_problem(t, P.probs, DgemmProblem{L.G + o2 * sp + o1, L.Cinv + o1 * sp + o1,
                                             L.tmp + q * b * b, sp, 1, sp, 1, b, rows, b, b, 1.0,
                                             0.0, 0});
      }
    }
    x.off = (int64_t)P.probs.size();
    for (const FactorLayout& L : Ls) {
      const int64_t sp = L.s_pad;
      if (b >= sp) continue;
      const int64_t full = sp / (2 * b);
      for (int64_t q = 0; q <= full; ++q) {
        const int64_t o1 = 2 * b * q, o2 = o1 + b, rows = std::min(b, sp - o2);
        if (rows <= 0) break;
        add_problem(x, P.probs, DgemmProblem{L.Cinv + o2 * sp + o2, L.tmp + q * b * b,
                                             L.Cinv + o2 * sp + o1, sp, 1, b, 1, sp, rows, b, rows,
                                             -1.0, 0.0, 0});
      }
    }
    P.levels.push_back(t);
    P.levels.push_back(x);
  }
}

struct SetupPlan {
  size_t slot = 0, own_total = 0;
  std::vector<size_t> own_off;
  size_t infos_off = 0, members_off = 0, probs_off = 0, total = 0;
  std::vector<FactorLayout> Ls;
  GroupedFactorPlan G;
};
// Workspace: k stream slots, every problem's own factor region, pivot flags, the member
// and GEMM descriptors. With base == nullptr only the sizes are formed.
void plan_setup(const krr_setup_problem* probs, int count, int k, char* base, SetupPlan& S) {
  S = SetupPlan{};
  std::vector<size_t> own(count);
  for (int i = 0; i < count; ++i) {
    size_t sl;
    setup_sizes(probs[i], sl, own[i]);
    S.slot = std::max(S.slot, sl);
  }
  size_t off = (size_t)k * S.slot;
  S.own_off.resize(count);
  S.Ls.resize(count);
  for (int i = 0; i < count; ++i) {
    S.own_off[i] = off;
    Bump scratch(nullptr), mine(base ? base + off : nullptr);
    layout_factor_parts(scratch, mine, S.Ls[i], probs[i].n, probs[i].s);
    off += own[i];
  }
  plan_grouped_factor(S.Ls, S.G);
  S.infos_off = off;
  off += (size_t)round_up((int64_t)count * (int64_t)sizeof(int), 256);
  S.members_off = off;
  off += (size_t)round_up((int64_t)count * (int64_t)sizeof(FactorMember), 256);
  S.probs_off = off;
  off += (size_t)round_up((int64_t)std::max<size_t>(S.G.probs.size(), 1) * (int64_t)sizeof(DgemmProblem), 256);
  S.total = off + 256;
}
bool setup_problem_ok(const krr_setup_problem& p) {
  return p.n >= 2 && p.s >= 1 && p.d >= 1 && p.s < p.n;
}
}  // namespace

size_t krr_setup_many_workspace_bytes(const krr_setup_problem* probs, int32_t count,
                                      int32_t nstreams) {
  if (!probs || count < 1) return 0;
  for (int i = 0; i < count; ++i)
    if (!setup_problem_ok(probs[i])) return 0;
  const int k = std::max(1, std::min<int32_t>(nstreams, KRR_SETUP_MAX_STREAMS));
  SetupPlan S;
  plan_setup(probs, count, k, nullptr, S);
  return S.total;
}

krr_status krr_setup_many(krr_setup_problem* probs, int32_t count, int32_t nstreams, void* ws,
                          size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!probs || count < 1) return fail(KRR_E_ARG, "krr_setup_many: no problems");
  for (int i = 0; i < count; ++i) {
    krr_setup_problem& p = probs[i];
    p.info = 0;
    if (!p.X || !p.W || !p.b || !p.Z || !p.C || !p.Ut)
      return fail(KRR_E_ARG, "krr_setup_many: problem %d: null pointer", i);
    if (p.n < 2 || p.d < 1 || p.s < 1 || p.s >= p.n || p.ldx < p.d || p.ldz < p.s || p.ldu < p.s)
      return fail(KRR_E_ARG, "krr_setup_many: problem %d: need 1 <= s < n, ld >= row length", i);
    if (!(p.lambda_p > 0.0) || !std::isfinite(p.lambda_p))
      return fail(KRR_E_ARG, "krr_setup_many: problem %d: lambda_p must be > 0", i);
  }
  const int k = std::max(1, std::min<int32_t>(nstreams, KRR_SETUP_MAX_STREAMS));
  const size_t need = krr_setup_many_workspace_bytes(probs, count, k);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  char* base = static_cast<char*>(ws);
  SetupPlan S;
  plan_setup(probs, count, k, base, S);
  int* infos = reinterpret_cast<int*>(base + S.infos_off);
  FactorMember* mem_d = reinterpret_cast<FactorMember*>(base + S.members_off);
  DgemmProblem* probs_d = reinterpret_cast<DgemmProblem*>(base + S.probs_off);
  std::vector<FactorMember> mem_h(count);
  for (int i = 0; i < count; ++i) mem_h[i] = FactorMember{S.Ls[i].G, S.Ls[i].Cinv, S.Ls[i].info, S.Ls[i].s_pad};
  hipStream_t st = (hipStream_t)stream;
  // streams at the default priority; they start after the work already on `stream` and the
  // caller's stream waits for all of them at the end of each phase
  std::vector<hipStream_t> ss(k, nullptr);
  std::vector<hipEvent_t> ev(k + 1, nullptr);
  auto cleanup = [&]() {
    for (auto& e : ev) if (e) (void)hipEventDestroy(e);
    for (auto& q : ss) if (q) (void)hipStreamDestroy(q);
  };
  auto fork = [&]() -> hipError_t {
    hipError_t e = hipEventRecord(ev[k], st);
    for (int j = 0; j < k && e == hipSuccess; ++j) e = hipStreamWaitEvent(ss[j], ev[k], 0);
    return e;
  };
  auto join = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (int j = 0; j < k && e == hipSuccess; ++j) {
      e = hipEventRecord(ev[j], ss[j]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[j], 0);
    }
    return e;
  };
  hipError_t e = hipSuccess;
  for (int j = 0; j <= k && e == hipSuccess; ++j) e = hipEventCreateWithFlags(&ev[j], hipEventDisableTiming);
  for (int j = 0; j < k && e == hipSuccess; ++j) e = hipStreamCreateWithFlags(&ss[j], hipStreamNonBlocking);
  // descriptors: the host vectors live until the synchronisation at the end
  if (e == hipSuccess) e = hipMemcpyAsync(mem_d, mem_h.data(), sizeof(FactorMember) * count, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !S.G.probs.empty())
    e = hipMemcpyAsync(probs_d, S.G.probs.data(), sizeof(DgemmProblem) * S.G.probs.size(),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = fill_i32(infos, count, 0, st);
  if (e == hipSuccess) e = fork();
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    cleanup();
    return fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e));
  }
  // largest problems first, each to the stream with the least estimated work so far
  std::vector<int> order(count), stream_of(count, 0);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto cost = [&](int i) { return (double)probs[i].n * (double)probs[i].s * (double)(probs[i].s + probs[i].d); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<double> load(k, 0.0);
  for (int i : order) {
    const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[j] += cost(i);
    stream_of[i] = j;
  }
  krr_status status = KRR_OK;
  // phase 1 (streams): features and Gram of every problem, scratch in the stream's slot
  for (int i : order) {
    krr_setup_problem& p = probs[i];
    const int j = stream_of[i];
    void* wsj = base + (size_t)j * S.slot;
    status = features_impl("krr_setup_many", p.X, p.n, p.d, p.ldx, p.W, p.s, p.b, p.s, p.Z, p.ldz,
                           wsj, S.slot, ss[j]);
    if (status != KRR_OK) break;
    Bump scratch(wsj), mine(base + S.own_off[i]);
    FactorLayout L;
    layout_factor_parts(scratch, mine, L, p.n, p.s);
    e = gram_form_async(p.Z, p.n, p.s, p.ldz, p.lambda_p, L, ss[j]);
    if (e != hipSuccess) { status = fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e)); break; }
  }
  e = join();
  if (e != hipSuccess && status == KRR_OK) status = fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e));
  // phase 2 (caller's stream): the grouped FP64 factor and inverse of all problems
  if (status == KRR_OK) {
    const GroupedFactorPlan& G = S.G;
    for (size_t t = 0; t < G.trail.size() && e == hipSuccess; ++t) {
      const GroupLaunch& g = G.trail[t];
      e = cholesky_step_grouped(mem_d, count, 64 * (int64_t)t, g.max_m, st);
      if (e == hipSuccess) e = dgemm_grouped(probs_d + g.off, (int)g.count, g.max_m, g.max_n, st);
    }
    if (e == hipSuccess) e = diag_inverse_grouped(mem_d, count, G.max_s_pad, st);
    for (size_t l = 0; l < G.levels.size() && e == hipSuccess; ++l) {
      const GroupLaunch& g = G.levels[l];
      e = dgemm_grouped(probs_d + g.off, (int)g.count, g.max_m, g.max_n, st);
    }
    if (e == hipSuccess) e = fork();
    if (e != hipSuccess) status = fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e));
  }
  // phase 3 (streams): C, the operand splits and Ut = Z C^{-T} of every problem
  if (status == KRR_OK) {
    for (int i : order) {
      krr_setup_problem& p = probs[i];
      const int j = stream_of[i];
      Bump scratch(base + (size_t)j * S.slot), mine(base + S.own_off[i]);
      FactorLayout L;
      layout_factor_parts(scratch, mine, L, p.n, p.s);
      e = hipMemcpyAsync(infos + i, L.info, sizeof(int), hipMemcpyDeviceToDevice, ss[j]);
      if (e == hipSuccess) e = factor_tail(L, p.Z, p.n, p.s, p.ldz, p.C, p.Ut, p.ldu, ss[j]);
      if (e != hipSuccess) { status = fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e)); break; }
    }
    e = join();
    if (e != hipSuccess && status == KRR_OK) status = fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e));
  }
  std::vector<int> h(count, 0);
  if (status == KRR_OK) {
    e = hipMemcpyAsync(h.data(), infos, sizeof(int) * count, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) status = fail(KRR_E_HIP, "krr_setup_many: %s", hipGetErrorString(e));
  } else {
    (void)join();
    (void)hipStreamSynchronize(st);
  }
  cleanup();
  if (status != KRR_OK) return status;
  int bad = -1;
  for (int i = 0; i < count; ++i) {
    probs[i].info = h[i];
    if (h[i] != 0 && bad < 0) bad = i;
  }
  if (bad >= 0)
    return fail(KRR_E_NOT_SPD, "krr_setup_many: problem %d: Z^T Z + lambda_p I not positive definite at pivot %d",
                bad, h[bad]);
  return KRR_OK;
}

// ---------------------------------------------------------------- precond apply
krr_status krr_precond_apply(const float* Ut, int64_t n, int64_t s, int64_t ldu, double lambda_p,
                             const double* R, int64_t m, int64_t ldr, double* Zout, int64_t ldz,
                             void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!Ut || !R || !Zout) return fail(KRR_E_ARG, "krr_precond_apply: null pointer");
  if (n < 2 || s < 1 || s >= n || ldu < s || m < 1 || ldr < m || ldz < m)
    return fail(KRR_E_ARG, "krr_precond_apply: need 1 <= s < n, m >= 1 and ld >= width");
  if (!(lambda_p > 0.0) || !std::isfinite(lambda_p))
    return fail(KRR_E_ARG, "krr_precond_apply: lambda_p must be > 0");
  if (static_cast<const void*>(R) == static_cast<const void*>(Zout))
    return fail(KRR_E_ARG, "krr_precond_apply: Zout must not alias R");
  CHECK_ST(check_ws(ws, ws_bytes, krr_workspace_bytes(KRR_OP_PRECOND_APPLY, n, n, 0, s, m, 0)));
  Bump bb(ws);
  ApplyLayout L;
  layout_apply(bb, L, n, s, m);
  hipStream_t st = (hipStream_t)stream;
  const double* r = R;
  if (ldr != m) {
    CHECK_HIP(copy2d(R, ldr, L.r, m, n, m, st));
    r = L.r;
  }
  double* z = ldz == m ? Zout : L.z;
  CHECK_HIP(precond_apply(Ut, ldu, n, s, m, lambda_p, r, z, L.part, L.nchunk, L.T, st));
  if (ldz != m) CHECK_HIP(copy2d(L.z, m, Zout, ldz, n, m, st));
  return KRR_OK;
}

// ---------------------------------------------------------------- kernel matmat
namespace {

// Kernel descriptor checks (Gaussian: sigma > 0; polynomial: degree 1..KRR_POLY_MAX_DEGREE,
// gamma >= 0, c >= 0, FP16X3 or FP64 products, no sigma-derivative).
krr_status check_kernel(const krr_kernel* k, int32_t prec, int32_t deriv, const char* fn) {
  if (!k) return fail(KRR_E_ARG, "%s: null kernel descriptor", fn);
  if (k->kind == KRR_KERNEL_GAUSSIAN) {
    if (!(k->sigma > 0.0) || !std::isfinite(k->sigma)) return fail(KRR_E_ARG, "%s: sigma must be > 0", fn);
    return KRR_OK;
  }
  if (k->kind != KRR_KERNEL_POLYNOMIAL) return fail(KRR_E_ARG, "%s: unknown kernel kind %d", fn, k->kind);
  if (k->degree < 1 || k->degree > KRR_POLY_MAX_DEGREE)
    return fail(KRR_E_ARG, "%s: polynomial degree must be in [1, %d]", fn, KRR_POLY_MAX_DEGREE);
  if (!(k->gamma >= 0.0) || !std::isfinite(k->gamma) || !(k->coef0 >= 0.0) || !std::isfinite(k->coef0))
    return fail(KRR_E_ARG, "%s: polynomial gamma and c must be finite and >= 0", fn);
  if (prec == KRR_PREC_BF16X3)
    return fail(KRR_E_ARG, "%s: polynomial kernel products use KRR_PREC_F16X3 or KRR_PREC_FP64", fn);
  if (deriv) return fail(KRR_E_ARG, "%s: deriv applies to the Gaussian kernel only", fn);
  return KRR_OK;
}

krr_status kernel_matmat_impl(const char* fn, const krr_kernel* kern, const float* X1, int64_t n1,
                              int64_t ldx1, const float* X2, int64_t n2, int64_t ldx2, int64_t d,
                              double shift, const double* V, int64_t m, int64_t ldv, double* OUT,
                              int64_t ldo, int32_t deriv, int32_t prec, void* ws, size_t ws_bytes,
                              void* stream) {
  g_err[0] = 0;
  if (!X1 || !X2 || !V || !OUT) return fail(KRR_E_ARG, "%s: null pointer", fn);
  if (n1 < 1 || n2 < 1 || d < 1 || m < 1 || ldx1 < d || ldx2 < d || ldv < m || ldo < m)
    return fail(KRR_E_ARG, "%s: bad sizes or strides", fn);
  CHECK_ST(check_kernel(kern, prec, deriv, fn));
  if (shift != 0.0 && n1 != n2) return fail(KRR_E_ARG, "%s: shift needs n1 == n2", fn);
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "%s: unknown precision %d", fn, prec);
  if (prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "%s: BF16X3 supports d <= 254 (d=%lld)", fn, (long long)d);
  const size_t need = krr_workspace_bytes(KRR_OP_KERNEL_MATMAT, n1, n2, d, 0, m, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  MatmatCtx c;
  // K(X, X) V with the same points on both sides: the square layout (the sizing above holds
  // for it: it shares the FP64 arrays and reserves the same column-side accumulator)
  const bool same = X1 == X2 && n1 == n2 && ldx1 == ldx2;
  layout_matmat(bb, c, n1, n2, d, m, prec, same, n1 == n2);
  float* Vf = prec != KRR_PREC_FP64 ? bb.take<float>(round_up(n2, ROW_PAD) * m) : nullptr;
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(prepare_points(c, X1, ldx1, same ? nullptr : X2, ldx2, *kern, st));
  if (Vf) {
    CHECK_HIP(vec_to_f32(V, n2, m, ldv, round_up(n2, ROW_PAD), m, Vf, st));
    CHECK_HIP(run_matmat(c, Vf, nullptr, m, deriv != 0, st));
  } else {
    CHECK_HIP(run_matmat(c, nullptr, V, ldv, deriv != 0, st));
  }
  CHECK_HIP(matmat_finalize<double>(c.part, c.part_stride, c.nsplit, n1, m, m, shift, V, ldv, OUT,
                                    ldo, st));
  return KRR_OK;
}

krr_kernel gaussian(double sigma) {
  krr_kernel k{};
  k.kind = KRR_KERNEL_GAUSSIAN;
  k.sigma = sigma;
  return k;
}

}  // namespace

krr_status krr_kernel_matmat(const float* X1, int64_t n1, int64_t ldx1, const float* X2, int64_t n2,
                             int64_t ldx2, int64_t d, double sigma, double shift, const double* V,
                             int64_t m, int64_t ldv, double* OUT, int64_t ldo, int32_t deriv,
                             int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  const krr_kernel k = gaussian(sigma);
  return kernel_matmat_impl("krr_kernel_matmat", &k, X1, n1, ldx1, X2, n2, ldx2, d, shift, V, m,
                            ldv, OUT, ldo, deriv, prec, ws, ws_bytes, stream);
}

krr_status krr_kernel_matmat_k(const krr_kernel* kernel, const float* X1, int64_t n1, int64_t ldx1,
                               const float* X2, int64_t n2, int64_t ldx2, int64_t d, double shift,
                               const double* V, int64_t m, int64_t ldv, double* OUT, int64_t ldo,
                               int32_t deriv, int32_t prec, void* ws, size_t ws_bytes,
                               void* stream) {
  return kernel_matmat_impl("krr_kernel_matmat_k", kernel, X1, n1, ldx1, X2, n2, ldx2, d, shift, V,
                            m, ldv, OUT, ldo, deriv, prec, ws, ws_bytes, stream);
}

// ------------------------------------------------------------------ autotuning
krr_status krr_autotune_matmat(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                               int64_t ldx, int64_t m, int32_t prec, krr_tune_report* rep,
                               void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !rep) return fail(KRR_E_ARG, "krr_autotune_matmat: null pointer");
  if (n < 1 || d < 1 || m < 1 || ldx < d) return fail(KRR_E_ARG, "krr_autotune_matmat: bad sizes");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_autotune_matmat: unknown precision %d", prec);
  CHECK_ST(check_kernel(kernel, prec, 0, "krr_autotune_matmat"));
  const size_t need = krr_workspace_bytes(KRR_OP_AUTOTUNE, n, n, d, 0, m, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  hipStream_t st = (hipStream_t)stream;
  Bump bb(ws);
  TuneLayout L;
  layout_tune(bb, L, n, d, m, prec);
  MatmatCtx& c = L.mm;
  const int64_t key_k = prec == KRR_PREC_FP64 ? c.dp : c.Kp;
  // the rule's choice (the table entry for this shape, if any, is ignored while timing)
  int ns0 = choose_nsplit(n, n);
  if (c.pv && c.Kp > 128 && ceil_div(n, 128) >= 64) ns0 = 8;
  const int w0 = (int)pv_pass_width(c.Kp);
  CHECK_HIP(prepare_points(c, X, ldx, nullptr, 0, *kernel, st));
  CHECK_HIP(hash_fill(L.V, n * m, 0x7e57, st));
  // candidates: the rule, fewer splits, and 8 splits (the grouped launch for large d); for
  // large d with more than 64 (32) right-hand sides also 64-column (32-column) passes
  std::vector<std::pair<int, int>> cand;
  auto add = [&](int ns, int w) {
    if (ns < 1 || ns > c.nsplit_max) return;
    for (auto& p : cand)
      if (p.first == ns && p.second == w) return;
    cand.push_back({ns, w});
  };
  std::vector<int> ws_opts = {w0};
  if (c.pv && c.Kp > 128 && m > 64) ws_opts.push_back(64);
  if (c.pv && c.Kp > 128 && m > 32) ws_opts.push_back(32);
  for (int w : ws_opts) {
    add(ns0, w);
    add(ns0 / 2, w);
    add(ns0 / 4, w);
    add(8, w);
  }
  hipEvent_t e0, e1;
  CHECK_HIP(hipEventCreate(&e0));
  CHECK_HIP(hipEventCreate(&e1));
  double best_ms = 1e30, def_ms = 0.0;
  int best = 0;
  hipError_t err = hipSuccess;
  for (size_t ci = 0; ci < cand.size() && err == hipSuccess; ++ci) {
    c.nsplit = cand[ci].first;
    c.pass_w = cand[ci].second;
    double tmin = 1e30;
    for (int rep_i = 0; rep_i < 4 && err == hipSuccess; ++rep_i) {
      if (prec != KRR_PREC_FP64)
        err = vec_to_f32(L.V, n, m, m, round_up(n, ROW_PAD), m, L.Vf, st);
      if (err == hipSuccess) err = hipEventRecord(e0, st);
      if (err == hipSuccess)
        err = prec == KRR_PREC_FP64 ? run_matmat(c, nullptr, L.V, m, false, st)
                                    : run_matmat(c, L.Vf, nullptr, m, false, st);
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float t = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
      if (rep_i > 0) tmin = std::min(tmin, (double)t);  // the first run warms up
    }
    if (ci == 0) def_ms = tmin;
    if (tmin < best_ms) { best_ms = tmin; best = (int)ci; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  CHECK_HIP(err);
  // keep the rule unless a candidate is clearly faster (timing noise must not flip it)
  if (best_ms > 0.97 * def_ms) { best = 0; best_ms = def_ms; }
  TuneChoice tc;
  tc.nsplit = cand[best].first;
  tc.pass_width = cand[best].second;
  tc.ms_default = def_ms;
  tc.ms_best = best_ms;
  tune_store(prec, 0, key_k, m, n, tc);
  rep->candidates = (int32_t)cand.size();
  rep->default_nsplit = cand[0].first;
  rep->default_pass_width = cand[0].second;
  rep->nsplit = tc.nsplit;
  rep->pass_width = tc.pass_width;
  rep->default_ms = def_ms;
  rep->best_ms = best_ms;
  return KRR_OK;
}

// ------------------------------------------------------------------------ PCG
namespace {

// Device time of the kernel products of one solve: HIP event pairs on the solve's stream,
// harvested at synchronisation points.
struct MMTimer {
  static constexpr int CAP = 32;
  hipEvent_t a[CAP], b[CAP];
  int used = 0, created = 0, calls = 0;
  double ms = 0.0;
  hipError_t init() {
    for (; created < CAP; ++created) {
      hipError_t e = hipEventCreate(&a[created]);
      if (e != hipSuccess) return e;
      e = hipEventCreate(&b[created]);
      if (e != hipSuccess) { (void)hipEventDestroy(a[created]); return e; }
    }
    return hipSuccess;
  }
  ~MMTimer() {
    for (int i = 0; i < created; ++i) { (void)hipEventDestroy(a[i]); (void)hipEventDestroy(b[i]); }
  }
  hipError_t harvest() {
    if (used == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(b[used - 1]);
    if (e != hipSuccess) return e;
    for (int i = 0; i < used; ++i) {
      float t = 0.0f;
      if ((e = hipEventElapsedTime(&t, a[i], b[i])) != hipSuccess) return e;
      ms += t;
    }
    used = 0;
    return hipSuccess;
  }
  hipError_t begin(hipStream_t st) {
    if (used == CAP) {
      hipError_t e = harvest();
      if (e != hipSuccess) return e;
    }
    return hipEventRecord(a[used], st);
  }
  hipError_t end(hipStream_t st) {
    hipError_t e = hipEventRecord(b[used], st);
    ++used;
    ++calls;
    return e;
  }
};

hipError_t timed_matmat(MMTimer* tm, const MatmatCtx& c, float* Vf, const double* V64,
                        int64_t ldv, bool deriv, hipStream_t st) {
  hipError_t e;
  if (tm && (e = tm->begin(st)) != hipSuccess) return e;
  if ((e = run_matmat(c, Vf, V64, ldv, deriv, st)) != hipSuccess) return e;
  return tm ? tm->end(st) : hipSuccess;
}

hipError_t fill2d_zero(double* a, int64_t lda, int64_t n, int64_t m, hipStream_t st) {
  if (lda == m) return fill_f64(a, n * m, 0.0, st);
  return fill2d_f64(a, lda, n, m, 0.0, st);  // strided: one launch over the n x m block
}

struct SolveArgs {
  PCGLayout* L;
  int64_t n, m, s, ldu;
  const float* Ut;
  double lambda, lambda_p, tol;
  int use_precond, max_iter, check_every;
  bool mixed;
  MMTimer* tm;
};

// One PCG run on A x = rhs (rhs n x m contiguous, x strided), starting from x.
// warm: x holds a starting point that is not zero. Returns iterations through *iters.
krr_status pcg_core(const SolveArgs& a, const double* rhs, int64_t ldr, double* x, int64_t ldx,
                    bool warm, int* iters, std::vector<double>* hist, hipStream_t st) {
  PCGLayout& L = *a.L;
  const int64_t n = a.n, m = a.m;
  CGScalars S{L.ynorm, L.rnorm, L.rho, L.alpha, L.beta, L.active, L.broken, L.col_iters, L.count};
  const int64_t ldpf = m;
  // r0 = rhs - A x0
  if (warm) {
    if (a.mixed) {
      CHECK_HIP(fill_f32(L.pf, round_up(n, ROW_PAD) * m, 0.0f, st));
      // FP32 copy of x for the product (row stride m)
      CHECK_HIP(copy2d(x, ldx, L.p, m, n, m, st));
      CHECK_HIP(cg_update_p(L.p, L.p, L.pf, ldpf, L.beta, L.active, 1, n, m, st));
      CHECK_HIP(timed_matmat(a.tm, L.mm, L.pf, nullptr, ldpf, false, st));
    } else {
      CHECK_HIP(copy2d(x, ldx, L.p, m, n, m, st));
      CHECK_HIP(timed_matmat(a.tm, L.mm, nullptr, L.p, m, false, st));
    }
    CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, a.lambda,
                                      L.p, m, L.ax, m, st));
    CHECK_HIP(residual_from(rhs, ldr, L.ax, n, m, L.r, st));
  } else {
    CHECK_HIP(residual_from(rhs, ldr, nullptr, n, m, L.r, st));
  }
  CHECK_HIP(dot_partial<double, double>(rhs, ldr, rhs, ldr, n, m, L.part_yy, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(L.r, m, L.r, m, n, m, L.part_rr, NBLK, st));
  if (a.use_precond) {
    CHECK_HIP(precond_apply(a.Ut, a.ldu, n, a.s, m, a.lambda_p, L.r, L.z, L.pc_part, L.nchunk, L.T, st));
    CHECK_HIP(dot_partial<double, double>(L.r, m, L.z, m, n, m, L.part_rz, NBLK, st));
  } else {
    CHECK_HIP(copy2d(L.r, m, L.z, m, n, m, st));
  }
  CHECK_HIP(cg_init_scalars(L.part_yy, L.part_rr, a.use_precond ? L.part_rz : nullptr, NBLK, m,
                            a.tol, S, st));
  CHECK_HIP(cg_update_p(L.z, L.p, a.mixed ? L.pf : nullptr, ldpf, L.beta, L.active, 1, n, m, st));
  int h_count = 0;
  CHECK_HIP(hipMemcpyAsync(&h_count, L.count, sizeof(int), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  int it = 0;
  while (h_count > 0 && it < a.max_iter) {
    ++it;
    // q = (K + lambda I) p
    if (a.mixed) {
      CHECK_HIP(timed_matmat(a.tm, L.mm, L.pf, nullptr, ldpf, false, st));
      CHECK_HIP(matmat_finalize<float>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, a.lambda,
                                       L.pf, ldpf, L.q, m, st));
      CHECK_HIP(dot_partial<float, double>(L.pf, ldpf, L.q, m, n, m, L.part_pq, NBLK, st));
    } else {
      CHECK_HIP(timed_matmat(a.tm, L.mm, nullptr, L.p, m, false, st));
      CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, a.lambda,
                                        L.p, m, L.q, m, st));
      CHECK_HIP(dot_partial<double, double>(L.p, m, L.q, m, n, m, L.part_pq, NBLK, st));
    }
    CHECK_HIP(cg_alpha(L.part_pq, NBLK, m, S, st));
    if (a.mixed)
      CHECK_HIP(cg_update_xr<float>(x, ldx, L.r, L.pf, ldpf, L.q, L.alpha, n, m, L.part_rr, NBLK, st));
    else
      CHECK_HIP(cg_update_xr<double>(x, ldx, L.r, L.p, m, L.q, L.alpha, n, m, L.part_rr, NBLK, st));
    CHECK_HIP(cg_conv(L.part_rr, NBLK, m, a.tol, it, S, L.hist, st));
    if (a.use_precond) {
      CHECK_HIP(precond_apply(a.Ut, a.ldu, n, a.s, m, a.lambda_p, L.r, L.z, L.pc_part, L.nchunk, L.T, st));
      CHECK_HIP(dot_partial<double, double>(L.r, m, L.z, m, n, m, L.part_rz, NBLK, st));
      CHECK_HIP(cg_beta(L.part_rz, nullptr, NBLK, m, S, st));
      CHECK_HIP(cg_update_p(L.z, L.p, a.mixed ? L.pf : nullptr, ldpf, L.beta, L.active, 0, n, m, st));
    } else {
      CHECK_HIP(cg_beta(nullptr, L.part_rr, NBLK, m, S, st));
      CHECK_HIP(cg_update_p(L.r, L.p, a.mixed ? L.pf : nullptr, ldpf, L.beta, L.active, 0, n, m, st));
    }
    if (it % a.check_every == 0 || it == a.max_iter) {
      double hv = 0.0;
      CHECK_HIP(hipMemcpyAsync(&h_count, L.count, sizeof(int), hipMemcpyDeviceToHost, st));
      CHECK_HIP(hipMemcpyAsync(&hv, L.hist, sizeof(double), hipMemcpyDeviceToHost, st));
      CHECK_HIP(hipStreamSynchronize(st));
      if (hist) hist->push_back(hv);
    }
  }
  *iters = it;
  return KRR_OK;
}

// FP64 true residual R = rhs - (K + lambda I) x into L.ax; per-column relative norms to host.
krr_status true_residual(PCGLayout& L, const SolveArgs& a, const double* Y, int64_t ldy,
                         const double* x, int64_t ldx, std::vector<double>& rel, hipStream_t st) {
  MatmatCtx& c = a.mixed ? L.mm64 : L.mm;
  const int64_t n = a.n, m = a.m;
  CHECK_HIP(copy2d(x, ldx, L.delta, m, n, m, st));
  CHECK_HIP(run_matmat(c, nullptr, L.delta, m, false, st));  // FP64 check: not timed
  CHECK_HIP(matmat_finalize<double>(c.part, c.part_stride, c.nsplit, n, m, m, a.lambda, L.delta, m,
                                    L.ax, m, st));
  CHECK_HIP(residual_from(Y, ldy, L.ax, n, m, L.rhs, st));
  CHECK_HIP(dot_partial<double, double>(L.rhs, m, L.rhs, m, n, m, L.part_rr, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(Y, ldy, Y, ldy, n, m, L.part_yy, NBLK, st));
  std::vector<double> prr(NBLK * m), pyy(NBLK * m);
  CHECK_HIP(hipMemcpyAsync(prr.data(), L.part_rr, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipMemcpyAsync(pyy.data(), L.part_yy, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  rel.assign(m, 0.0);
  for (int64_t c2 = 0; c2 < m; ++c2) {
    double rr = 0.0, yy = 0.0;
    for (int b = 0; b < NBLK; ++b) { rr += prr[b * m + c2]; yy += pyy[b * m + c2]; }
    rel[c2] = yy > 0.0 ? std::sqrt(rr) / std::sqrt(yy) : std::sqrt(rr);
  }
  return KRR_OK;
}

}  // namespace

namespace {
krr_status pcg_solve_impl(const krr_kernel* kern, const float* X, int64_t n, int64_t d,
                          int64_t ldx, double lambda, const float* Ut, int64_t s, int64_t ldu,
                          const double* Y, int64_t ldy, double* alpha, int64_t lda, int64_t m,
                          const krr_pcg_opts* opts, krr_pcg_report* rep, void* ws,
                          size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  krr_pcg_opts o;
  krr_pcg_defaults(&o);
  if (opts) o = *opts;
  if (!X || !Y || !alpha) return fail(KRR_E_ARG, "krr_pcg_solve: null pointer");
  if (n < 1 || d < 1 || m < 1 || ldx < d || ldy < m || lda < m)
    return fail(KRR_E_ARG, "krr_pcg_solve: bad sizes or strides");
  CHECK_ST(check_kernel(kern, o.prec, 0, "krr_pcg_solve"));
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(KRR_E_ARG, "krr_pcg_solve: lambda must be > 0");
  if (!(o.tol > 0.0)) return fail(KRR_E_ARG, "krr_pcg_solve: tol must be > 0");
  if (o.max_iter < 1) return fail(KRR_E_ARG, "krr_pcg_solve: max_iter must be >= 1");
  if (!prec_ok(o.prec)) return fail(KRR_E_ARG, "krr_pcg_solve: unknown precision %d", o.prec);
  if (o.prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "krr_pcg_solve: BF16X3 supports d <= 254 (d=%lld)", (long long)d);
  if (o.use_precond) {
    if (!Ut || s < 1 || s >= n || ldu < s)
      return fail(KRR_E_ARG, "krr_pcg_solve: preconditioner needs Ut with 1 <= s < n, ldu >= s");
  } else {
    s = 0;
  }
  if (o.check_every < 1) o.check_every = 1;
  const double lambda_p = o.lambda_p > 0.0 ? o.lambda_p : lambda;
  const size_t need = krr_workspace_bytes(KRR_OP_PCG_SOLVE, n, n, d, s, m, o.prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  PCGLayout L;
  layout_pcg(bb, L, n, d, s, m, o.prec);
  hipStream_t st = (hipStream_t)stream;
  const bool mixed = o.prec != KRR_PREC_FP64;
  CHECK_HIP(prepare_points(L.mm, X, ldx, nullptr, 0, *kern, st));
  if (mixed && (o.true_residual || o.refine > 0))
    CHECK_HIP(prepare_points(L.mm64, X, ldx, nullptr, 0, *kern, st));

  MMTimer timer;
  CHECK_HIP(timer.init());
  SolveArgs a{&L, n, m, s, ldu, Ut, lambda, lambda_p, o.tol, o.use_precond, o.max_iter,
              o.check_every, mixed, &timer};
  std::vector<double> hist;
  int iters = 0;
  if (!o.warm_start) CHECK_HIP(fill2d_zero(alpha, lda, n, m, st));
  CHECK_ST(pcg_core(a, Y, ldy, alpha, lda, o.warm_start != 0, &iters, &hist, st));
  int total_iters = iters;
  std::vector<int> h_broken(m);
  std::vector<double> h_rnorm(m), h_ynorm(m);
  auto fetch = [&]() -> krr_status {
    CHECK_HIP(hipMemcpyAsync(h_broken.data(), L.broken, sizeof(int) * m, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipMemcpyAsync(h_rnorm.data(), L.rnorm, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipMemcpyAsync(h_ynorm.data(), L.ynorm, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipStreamSynchronize(st));
    return KRR_OK;
  };
  CHECK_ST(fetch());
  std::vector<int> broken0 = h_broken;
  std::vector<double> rel_rec(m), rel_true;
  for (int64_t c = 0; c < m; ++c) rel_rec[c] = h_ynorm[c] > 0 ? h_rnorm[c] / h_ynorm[c] : h_rnorm[c];
  int refine_steps = 0;
  if (o.true_residual || o.refine > 0) {
    CHECK_ST(true_residual(L, a, Y, ldy, alpha, lda, rel_true, st));
    while (refine_steps < o.refine) {
      double worst = 0.0;
      for (double v : rel_true) worst = std::max(worst, v);
      if (!(worst > o.tol)) break;
      // correction: A delta = R, R = Y - A alpha (in L.rhs); inner tolerance relative to R
      ++refine_steps;
      SolveArgs ai = a;
      ai.tol = std::max(0.5 * o.tol / worst, 1e-14);
      CHECK_HIP(copy2d(L.rhs, m, L.delta, m, n, m, st));  // keep R
      CHECK_HIP(fill_f64(L.ax, n * m, 0.0, st));
      // solve into L.ax (zero start), rhs = R (held in L.delta while L.rhs is reused)
      int it2 = 0;
      CHECK_ST(pcg_core(ai, L.delta, m, L.ax, m, false, &it2, &hist, st));
      total_iters += it2;
      CHECK_HIP(add2d(L.ax, m, alpha, lda, n, m, st));
      CHECK_ST(true_residual(L, a, Y, ldy, alpha, lda, rel_true, st));
    }
  }
  CHECK_HIP(timer.harvest());
  int conv = 0, brk = 0;
  for (int64_t c = 0; c < m; ++c) {
    if (broken0[c]) ++brk;
    if (!broken0[c] && rel_rec[c] <= o.tol) ++conv;
  }
  if (rep) {
    rep->iters = total_iters;
    rep->converged_cols = conv;
    rep->breakdown_cols = brk;
    rep->refine_steps = refine_steps;
    if (rep->relres_rec) for (int64_t c = 0; c < m; ++c) rep->relres_rec[c] = rel_rec[c];
    if (rep->relres_true)
      for (int64_t c = 0; c < m; ++c) rep->relres_true[c] = rel_true.empty() ? NAN : rel_true[c];
    int hl = 0;
    if (rep->history && rep->history_cap > 0)
      for (; hl < rep->history_cap && hl < (int)hist.size(); ++hl) rep->history[hl] = hist[hl];
    rep->history_len = hl;
    rep->matmat_calls = timer.calls;
    rep->matmat_ms = timer.ms;
  }
  if (brk > 0) return fail(KRR_E_BREAKDOWN, "krr_pcg_solve: %d column(s) broke down", brk);
  bool ok;
  if (refine_steps > 0) {
    ok = true;
    for (double v : rel_true) ok = ok && v <= o.tol;
  } else {
    ok = conv == m;
  }
  if (!ok) return fail(KRR_E_NO_CONV, "krr_pcg_solve: not converged after %d iterations", total_iters);
  return KRR_OK;
}
}  // namespace

krr_status krr_pcg_solve(const float* X, int64_t n, int64_t d, int64_t ldx, double sigma,
                         double lambda, const float* Ut, int64_t s, int64_t ldu, const double* Y,
                         int64_t ldy, double* alpha, int64_t lda, int64_t m,
                         const krr_pcg_opts* opts, krr_pcg_report* rep, void* ws, size_t ws_bytes,
                         void* stream) {
  const krr_kernel k = gaussian(sigma);
  return pcg_solve_impl(&k, X, n, d, ldx, lambda, Ut, s, ldu, Y, ldy, alpha, lda, m, opts, rep,
                        ws, ws_bytes, stream);
}

krr_status krr_pcg_solve_k(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                           int64_t ldx, double lambda, const float* Ut, int64_t s, int64_t ldu,
                           const double* Y, int64_t ldy, double* alpha, int64_t lda, int64_t m,
                           const krr_pcg_opts* opts, krr_pcg_report* rep, void* ws,
                           size_t ws_bytes, void* stream) {
  return pcg_solve_impl(kernel, X, n, d, ldx, lambda, Ut, s, ldu, Y, ldy, alpha, lda, m, opts, rep,
                        ws, ws_bytes, stream);
}

// -------------------------------------------------------------- TensorSketch
krr_status krr_tensorsketch(const float* X, int64_t n, int64_t d, int64_t ldx, double gamma,
                            double coef0, int32_t degree, const int32_t* hash, const float* sign,
                            int64_t s, float* Z, int64_t ldz, void* stream) {
  g_err[0] = 0;
  if (!X || !hash || !sign || !Z) return fail(KRR_E_ARG, "krr_tensorsketch: null pointer");
  if (n < 1 || d < 1 || ldx < d || ldz < s) return fail(KRR_E_ARG, "krr_tensorsketch: bad sizes or strides");
  if (degree < 1 || degree > KRR_POLY_MAX_DEGREE)
    return fail(KRR_E_ARG, "krr_tensorsketch: degree must be in [1, %d]", KRR_POLY_MAX_DEGREE);
  if (!(gamma >= 0.0) || !std::isfinite(gamma) || !(coef0 >= 0.0) || !std::isfinite(coef0))
    return fail(KRR_E_ARG, "krr_tensorsketch: gamma and c must be finite and >= 0");
  if (s < 2 || s > KRR_TENSORSKETCH_MAX_S || (s & (s - 1)))
    return fail(KRR_E_ARG, "krr_tensorsketch: s must be a power of two in [2, %d]",
                KRR_TENSORSKETCH_MAX_S);
  int logs = 0;
  while ((int64_t(1) << logs) < s) ++logs;
  CHECK_HIP(tensor_sketch(X, n, d, ldx, gamma, coef0, degree, hash, sign, logs, Z, ldz,
                          (hipStream_t)stream));
  return KRR_OK;
}

// ---------------------------------------------------- multiple-level sketching (Alg. 2)
krr_status krr_srht(const float* Z1, int64_t n, int64_t s1, int64_t ldz1, const float* signs,
                    const int32_t* sample, int64_t s2, float* Z2, int64_t ldz2, void* stream) {
  g_err[0] = 0;
  if (!Z1 || !signs || !sample || !Z2) return fail(KRR_E_ARG, "krr_srht: null pointer");
  if (n < 1 || s1 < 1 || s2 < 1 || ldz1 < s1 || ldz2 < s2)
    return fail(KRR_E_ARG, "krr_srht: bad sizes or strides");
  int64_t p = 1;
  while (p < s1) p *= 2;
  if (p > KRR_SRHT_MAX_S1)
    return fail(KRR_E_ARG, "krr_srht: s1 padded to a power of two must be <= %d", KRR_SRHT_MAX_S1);
  if (s2 > p) return fail(KRR_E_ARG, "krr_srht: s2 must not exceed the padded s1 (%lld)", (long long)p);
  CHECK_HIP(srht_rows(Z1, n, s1, ldz1, signs, sample, s2, Z2, ldz2, (hipStream_t)stream));
  return KRR_OK;
}

krr_status krr_gaussian_project(const float* Z2, int64_t n, int64_t s2, int64_t ldz2,
                                const float* S3, int64_t s3, float* Z3, int64_t ldz3, void* ws,
                                size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!Z2 || !S3 || !Z3) return fail(KRR_E_ARG, "krr_gaussian_project: null pointer");
  if (n < 1 || s2 < 1 || s3 < 1 || ldz2 < s2 || ldz3 < s3)
    return fail(KRR_E_ARG, "krr_gaussian_project: bad sizes or strides");
  const size_t need = krr_workspace_bytes(KRR_OP_GAUSSIAN_PROJECT, n, n, s2, s3, 0, KRR_PREC_F16X3);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  ProjLayout L;
  layout_project(bb, L, n, s2, s3);
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(fill_f32(L.stats, 4, 0.0f, st));
  CHECK_HIP(absmax<float>(Z2, n, s2, ldz2, L.stats + 0, st));
  CHECK_HIP(absmax<float>(S3, s3, s2, s2, L.stats + 1, st));
  CHECK_HIP((split_operand<float, _Float16>(Z2, n, s2, ldz2, L.stats + 0, 0, L.np, L.kp, L.Ah, L.Al, st)));
  CHECK_HIP((split_operand<float, _Float16>(S3, s3, s2, s2, L.stats + 1, 0, L.sp, L.kp, L.Bh, L.Bl, st)));
  SplitOperand A{L.Ah, L.Al, L.kp, L.stats + 0}, B{L.Bh, L.Bl, L.kp, L.stats + 1};
  CHECK_HIP(gemm_nt_f16x3(A, B, n, s3, L.kp, 1, EPI_F32, 0, 0, 1.0 / std::sqrt((double)s3),
                          nullptr, 0, Z3, ldz3, nullptr, 1.0f, st));
  return KRR_OK;
}

// ------------------------------------------ preconditioner test and adaptive sketch size
namespace {

// dot products <a, b> (and optionally <c, d>) of n-vectors, summed on the host in fixed order
krr_status dots(const double* a, const double* b, const double* c, const double* d, int64_t n,
                double* part, double* r1, double* r2, hipStream_t st) {
  CHECK_HIP((dot_partial<double, double>(a, 1, b, 1, n, 1, part, NBLK, st)));
  if (c) CHECK_HIP((dot_partial<double, double>(c, 1, d, 1, n, 1, part + NBLK, NBLK, st)));
  double h[2 * NBLK];
  CHECK_HIP(hipMemcpyAsync(h, part, sizeof(double) * (c ? 2 : 1) * NBLK, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  double s1 = 0.0, s2 = 0.0;
  for (int i = 0; i < NBLK; ++i) s1 += h[i];
  if (c)
    for (int i = 0; i < NBLK; ++i) s2 += h[NBLK + i];
  *r1 = s1;
  if (r2) *r2 = s2;
  return KRR_OK;
}

// out = K v (the kernel alone) with the test's one-column product
krr_status kernel_vec(TestLayout& L, const double* v, double* out, int64_t n, hipStream_t st) {
  if (L.mm.prec == KRR_PREC_FP64) {
    CHECK_HIP(run_matmat(L.mm, nullptr, v, 1, false, st));
  } else {
    CHECK_HIP(vec_to_f32(v, n, 1, 1, round_up(n, ROW_PAD), 1, L.vf, st));
    CHECK_HIP(run_matmat(L.mm, L.vf, nullptr, 1, false, st));
  }
  CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, 1, 1, 0.0,
                                    (const double*)nullptr, 1, out, 1, st));
  return KRR_OK;
}

krr_status precond_test_impl(const krr_kernel* kern, const float* X, int64_t n, int64_t d,
                             int64_t ldx, const float* Z, int64_t s, int64_t ldz, double lambda,
                             int32_t iters, int32_t prec, krr_precond_test_report* rep, void* ws,
                             hipStream_t st) {
  Bump bb(ws);
  TestLayout L;
  layout_test(bb, L, n, d, s, prec);
  // eigen-decomposition of Z^T Z through the Cholesky factor of Z^T Z + jitter I. The Gram
  // is formed in FP64 from the exact FP64 values of Z (products of FP32 numbers are exact),
  // so its rounding (~1e-16 ||G||) stays far below the jitter, which is far below the
  // threshold and is subtracted from the eigenvalues again.
  const double thr = 0.05 * lambda, jitter = 1e-4 * thr;
  CHECK_HIP(f32_to_f64_2d(Z, n, s, ldz, L.Zd, st));
  CHECK_HIP(dgemm(s, s, n, 1.0, L.Zd, 1, s, 0, L.Zd, s, 1, 0, 0.0, L.F.part, s, 0, 1, 1, st));
  CHECK_HIP(gram_finalize(L.F.part, 1, s, s, s * s, jitter, L.F.s_pad, L.F.G, st));
  CHECK_HIP(fill_i32(L.F.info, 1, 0, st));
  CHECK_HIP(fill_f64(L.F.Cinv, L.F.s_pad * L.F.s_pad, 0.0, st));
  CHECK_HIP(cholesky_blocked(L.F.G, L.F.s_pad, L.F.Cinv, L.F.info, st));
  int hinfo = 0;
  CHECK_HIP(hipMemcpyAsync(&hinfo, L.F.info, sizeof(int), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  if (hinfo != 0)
    return fail(KRR_E_NOT_SPD, "krr_precond_test: Z^T Z + jitter not positive definite at pivot %d "
                "(non-finite Z?)", hinfo);
  CHECK_HIP(copy_lower(L.F.G, L.F.s_pad, s, L.A, st));
  int sweeps = 0;
  CHECK_HIP(jacobi_eig(L.A, (int)s, L.Vt, L.ev, L.off, 1e-14, 40, &sweeps, st));
  std::vector<double> ev(s);
  CHECK_HIP(hipMemcpyAsync(ev.data(), L.ev, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  // P projects on the eigenvectors of Z Z^T with eigenvalue above 0.05 lambda (Thm. 4):
  // u_i = Z v_i / sqrt(e_i) with e_i the eigenvalue of Z^T Z
  std::vector<int> idx;
  std::vector<double> sc, w;
  for (int64_t i = 0; i < s; ++i) {
    const double e = ev[i] - jitter;
    if (e > thr) {
      idx.push_back((int)i);
      sc.push_back(1.0 / std::sqrt(e));
      w.push_back(1.0 / std::sqrt(e));
    }
  }
  const int k = (int)idx.size();
  rep->rank = k;
  rep->jacobi_sweeps = sweeps;
  rep->power_iters = iters;
  if (k > 0) {
    CHECK_HIP(hipMemcpyAsync(L.idx, idx.data(), sizeof(int) * k, hipMemcpyHostToDevice, st));
    CHECK_HIP(hipMemcpyAsync(L.scale, sc.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
    CHECK_HIP(gather_scaled_rows(L.Vt, (int)s, L.idx, L.scale, k, L.Bk, st));
    // U_k = Z Bk^T (n x k, leading dimension s) on the split MFMA GEMM
    FactorLayout& F = L.F;
    CHECK_HIP(fill_f32(F.stats, 4, 0.0f, st));
    CHECK_HIP(absmax<float>(Z, n, s, ldz, F.stats + 0, st));
    CHECK_HIP(absmax<float>(L.Bk, k, s, s, F.stats + 1, st));
    CHECK_HIP((split_operand<float, _Float16>(Z, n, s, ldz, F.stats + 0, 0, F.np, F.sk, F.h1, F.l1, st)));
    CHECK_HIP((split_operand<float, _Float16>(L.Bk, k, s, s, F.stats + 1, 0, F.sp64, F.sk, F.ch, F.cl, st)));
    SplitOperand A{F.h1, F.l1, F.sk, F.stats + 0}, B{F.ch, F.cl, F.sk, F.stats + 1};
    CHECK_HIP(gemm_nt_f16x3(A, B, n, k, F.sk, 1, EPI_F32, 0, 0, 1.0, nullptr, 0, L.Uk, s, nullptr,
                            0.0f, st));
    // the weights 1 / sqrt(e_i) of condition 2 go to the device (reuse the scale array)
  }
  CHECK_HIP(prepare_points(L.mm, X, ldx, nullptr, 0, *kern, st));
  // condition 1: power iteration on (I - P) K (I - P)
  double num = 0.0, den = 0.0, mu1 = 0.0;
  CHECK_HIP(hash_fill(L.v, n, 0x5eed, st));
  for (int it = 0; it < iters; ++it) {
    const double* pv = L.v;
    if (k > 0) {
      CHECK_HIP(precond_apply(L.Uk, s, n, k, 1, 1.0, L.v, L.t, L.pc_part, L.nchunk, L.T, st));
      pv = L.t;
    }
    CHECK_ST(kernel_vec(L, pv, L.w, n, st));
    double* pw = L.w;
    if (k > 0) {
      CHECK_HIP(precond_apply(L.Uk, s, n, k, 1, 1.0, L.w, L.v, L.pc_part, L.nchunk, L.T, st));
      pw = L.v;
    }
    CHECK_ST(dots(pv, pw, pw, pw, n, L.part, &num, &den, st));
    double vv = 0.0;
    CHECK_ST(dots(pv, pv, nullptr, nullptr, n, L.part, &vv, nullptr, st));
    mu1 = vv > 0.0 ? num / vv : 0.0;
    if (!(den > 0.0)) break;
    CHECK_HIP(axpby(n, 1.0 / std::sqrt(den), pw, 0.0, nullptr, L.v, st));
  }
  rep->cond1 = mu1;
  // condition 2: extreme eigenvalues of B = W U_k^T K U_k W, W = diag(1 / sqrt(e_i)), by power
  // iteration on B and on mu_hi I - B
  double hi = 1.0, lo = 1.0;
  if (k > 0) {
    CHECK_HIP(hipMemcpyAsync(L.scale, w.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
    for (int pass = 0; pass < 2; ++pass) {
      CHECK_HIP(hash_fill(L.x, k, 0x5eed + 17 * (pass + 1), st));
      double mu = 0.0;
      for (int it = 0; it < iters; ++it) {
        CHECK_HIP(gemv_n(L.Uk, s, n, k, L.x, L.scale, L.t, st));
        CHECK_ST(kernel_vec(L, L.t, L.w, n, st));
        CHECK_HIP(gemv_t(L.Uk, s, n, k, L.w, L.scale, L.y, L.gpart, st));
        if (pass == 1) CHECK_HIP(axpby(k, hi, L.x, -1.0, L.y, L.y, st));  // (hi I - B) x
        double xy = 0.0, xx = 0.0, yy = 0.0;
        CHECK_ST(dots(L.x, L.y, L.x, L.x, k, L.part, &xy, &xx, st));
        CHECK_ST(dots(L.y, L.y, nullptr, nullptr, k, L.part, &yy, nullptr, st));
        mu = xx > 0.0 ? xy / xx : 0.0;
        if (!(yy > 0.0)) break;
        CHECK_HIP(axpby(k, 1.0 / std::sqrt(yy), L.y, 0.0, nullptr, L.x, st));
      }
      if (pass == 0) hi = mu;
      else lo = hi - mu;
    }
  }
  rep->ratio_lo = lo;
  rep->ratio_hi = hi;
  rep->passed = (rep->cond1 <= 0.1 * lambda && lo >= 0.9 && hi <= 1.1) ? 1 : 0;
  return KRR_OK;
}

}  // namespace

krr_status krr_precond_test(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                            int64_t ldx, const float* Z, int64_t s, int64_t ldz, double lambda,
                            int32_t power_iters, int32_t prec, krr_precond_test_report* rep,
                            void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !Z || !rep) return fail(KRR_E_ARG, "krr_precond_test: null pointer");
  if (n < 2 || d < 1 || s < 1 || s >= n || ldx < d || ldz < s)
    return fail(KRR_E_ARG, "krr_precond_test: need 1 <= s < n, ldx >= d, ldz >= s");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(KRR_E_ARG, "krr_precond_test: lambda must be > 0");
  if (power_iters < 1) return fail(KRR_E_ARG, "krr_precond_test: power_iters must be >= 1");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_precond_test: unknown precision %d", prec);
  CHECK_ST(check_kernel(kernel, prec, 0, "krr_precond_test"));
  const size_t need = krr_workspace_bytes(KRR_OP_PRECOND_TEST, n, n, d, s, 0, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  *rep = krr_precond_test_report{};
  return precond_test_impl(kernel, X, n, d, ldx, Z, s, ldz, lambda, power_iters, prec, rep, ws,
                           (hipStream_t)stream);
}

krr_status krr_adaptive_features(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                                 int64_t ldx, double lambda, const float* W, const float* b,
                                 const int32_t* hash, const float* sign, int64_t s0,
                                 int64_t s_max, float* Z, int64_t ldz, int64_t* s_out,
                                 krr_precond_test_report* history, int32_t history_cap,
                                 int32_t* history_len, int32_t power_iters, int32_t prec, void* ws,
                                 size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !Z || !s_out || !kernel) return fail(KRR_E_ARG, "krr_adaptive_features: null pointer");
  if (n < 2 || d < 1 || ldx < d || s0 < 1 || s_max < s0 || s_max >= n || ldz < s_max)
    return fail(KRR_E_ARG, "krr_adaptive_features: need 1 <= s0 <= s_max < n, ldz >= s_max");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(KRR_E_ARG, "krr_adaptive_features: lambda must be > 0");
  if (power_iters < 1) return fail(KRR_E_ARG, "krr_adaptive_features: power_iters must be >= 1");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_adaptive_features: unknown precision %d", prec);
  CHECK_ST(check_kernel(kernel, prec, 0, "krr_adaptive_features"));
  const bool poly = kernel->kind == KRR_KERNEL_POLYNOMIAL;
  if (poly ? (!hash || !sign) : (!W || !b))
    return fail(KRR_E_ARG, "krr_adaptive_features: the kernel's feature draw is missing");
  if (poly) {
    for (int64_t t = s0; t <= s_max; t *= 2)
      if ((t & (t - 1)) || t > KRR_TENSORSKETCH_MAX_S)
        return fail(KRR_E_ARG, "krr_adaptive_features: TensorSketch sizes must be powers of two <= %d",
                    KRR_TENSORSKETCH_MAX_S);
  }
  const size_t need = krr_workspace_bytes(KRR_OP_ADAPTIVE_FEATURES, n, n, d, s_max, 0, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  hipStream_t st = (hipStream_t)stream;
  int32_t len = 0;
  int64_t s = s0;
  for (;;) {
    // the first s features of the draw (Gaussian: columns of W and entries of b; polynomial:
    // the same hashes reduced modulo s)
    if (poly) {
      int logs = 0;
      while ((int64_t(1) << logs) < s) ++logs;
      CHECK_HIP(tensor_sketch(X, n, d, ldx, kernel->gamma, kernel->coef0, kernel->degree, hash,
                              sign, logs, Z, ldz, st));
    } else {
      CHECK_ST(features_impl("krr_adaptive_features", X, n, d, ldx, W, s_max, b, s, Z, ldz, ws,
                             ws_bytes, st));
    }
    krr_precond_test_report r{};
    CHECK_ST(precond_test_impl(kernel, X, n, d, ldx, Z, s, ldz, lambda, power_iters, prec, &r, ws, st));
    if (history && len < history_cap) history[len] = r;
    ++len;
    if (r.passed || 2 * s > s_max) break;
    s *= 2;
  }
  if (history_len) *history_len = len;
  *s_out = s;
  return KRR_OK;
}

// ------------------------------------------------------------------------ grad
krr_status krr_grad(const float* X, int64_t n, int64_t d, int64_t ldx, double sigma,
                    const double* alpha, const double* abar, int64_t m, int64_t ld,
                    double* dL_dsigma, double* dL_dlambda, int32_t prec, void* ws, size_t ws_bytes,
                    void* stream) {
  g_err[0] = 0;
  if (!X || !alpha || !abar || !dL_dsigma || !dL_dlambda) return fail(KRR_E_ARG, "krr_grad: null pointer");
  if (n < 1 || d < 1 || m < 1 || ldx < d || ld < m) return fail(KRR_E_ARG, "krr_grad: bad sizes");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(KRR_E_ARG, "krr_grad: sigma must be > 0");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_grad: unknown precision %d", prec);
  if (prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "krr_grad: BF16X3 supports d <= 254 (d=%lld)", (long long)d);
  const size_t need = krr_workspace_bytes(KRR_OP_GRAD, n, n, d, 0, m, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  GradLayout L;
  layout_grad(bb, L, n, d, m, prec);
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(prepare_points(L.mm, X, ldx, nullptr, 0, sigma, st));
  // W = (dK/dsigma) alpha
  if (prec == KRR_PREC_FP64) {
    CHECK_HIP(run_matmat(L.mm, nullptr, alpha, ld, true, st));
  } else {
    CHECK_HIP(vec_to_f32(alpha, n, m, ld, round_up(n, ROW_PAD), m, L.af, st));
    CHECK_HIP(run_matmat(L.mm, L.af, nullptr, m, true, st));
  }
  CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, 0.0, alpha,
                                    ld, L.w, m, st));
  CHECK_HIP(dot_partial<double, double>(abar, ld, L.w, m, n, m, L.part, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(abar, ld, alpha, ld, n, m, L.part + NBLK * m, NBLK, st));
  std::vector<double> h(2 * NBLK * m);
  CHECK_HIP(hipMemcpyAsync(h.data(), L.part, sizeof(double) * 2 * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  double s1 = 0.0, s2 = 0.0;
  for (int64_t e = 0; e < NBLK * m; ++e) { s1 += h[e]; s2 += h[NBLK * m + e]; }
  *dL_dsigma = -s1;
  *dL_dlambda = -s2;
  return KRR_OK;
}

// --------------------------------------------------- direct sigma-term of a loss
krr_status krr_kernel_dsigma_inner(const float* X1, int64_t n1, int64_t ldx1, const float* X2,
                                   int64_t n2, int64_t ldx2, int64_t d, double sigma,
                                   const double* V, int64_t m, int64_t ldv, const double* G,
                                   int64_t ldg, double* out, int32_t prec, void* ws,
                                   size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X1 || !X2 || !V || !G || !out) return fail(KRR_E_ARG, "krr_kernel_dsigma_inner: null pointer");
  if (n1 < 1 || n2 < 1 || d < 1 || m < 1 || ldx1 < d || ldx2 < d || ldv < m || ldg < m)
    return fail(KRR_E_ARG, "krr_kernel_dsigma_inner: bad sizes or strides");
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return fail(KRR_E_ARG, "krr_kernel_dsigma_inner: sigma must be > 0");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_kernel_dsigma_inner: unknown precision %d", prec);
  if (prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "krr_kernel_dsigma_inner: BF16X3 supports d <= 254 (d=%lld)", (long long)d);
  const size_t need = krr_workspace_bytes(KRR_OP_DSIGMA_INNER, n1, n2, d, 0, m, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  InnerLayout L;
  layout_inner(bb, L, n1, n2, d, m, prec);
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(prepare_points(L.mm, X1, ldx1, X2, ldx2, sigma, st));
  // W = (dK/dsigma) V, then <G, W> in FP64
  if (prec == KRR_PREC_FP64) {
    CHECK_HIP(run_matmat(L.mm, nullptr, V, ldv, true, st));
  } else {
    CHECK_HIP(vec_to_f32(V, n2, m, ldv, round_up(n2, ROW_PAD), m, L.vf, st));
    CHECK_HIP(run_matmat(L.mm, L.vf, nullptr, m, true, st));
  }
  CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n1, m, m, 0.0, V,
                                    ldv, L.w, m, st));
  CHECK_HIP(dot_partial<double, double>(G, ldg, L.w, m, n1, m, L.part, NBLK, st));
  std::vector<double> h(NBLK * m);
  CHECK_HIP(hipMemcpyAsync(h.data(), L.part, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  double acc = 0.0;
  for (int64_t e = 0; e < NBLK * m; ++e) acc += h[e];
  *out = acc;
  return KRR_OK;
}

}  // extern "C"

// =================================================================== batched plans
#include "batch.hpp"

struct krr_batch_plan {
  int count = 0, M = 0;
  int64_t N = 0;  // packed rows
  krr_pcg_opts opts{};
  std::vector<krr_batch_problem> probs;
  std::vector<BatchMeta> meta_h;
  std::vector<void*> allocs;
  // device arrays
  BatchMeta* meta = nullptr;
  int* row_inst = nullptr;
  BatchInst* inst = nullptr;
  BatchItem* items = nullptr;
  int nitems = 0, grid = 0, tiles_per_item = 0;
  int* counter = nullptr;
  int *live_list = nullptr, *live_count = nullptr, *chunk_cnt = nullptr;  // compacted queue
  RedItem* red = nullptr;
  int nred = 0;
  PCItem* pitems = nullptr;
  int npitems = 0;
  ZItem* zitems = nullptr;
  int nzitems = 0;
  int64_t smax = 0;
  float* pf = nullptr;
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *part_yy = nullptr, *part_rr = nullptr, *part_pq = nullptr, *part_rz = nullptr;
  double *pc_part = nullptr, *T = nullptr, *kpart = nullptr;
  float *colmax = nullptr, *vscale = nullptr;
  _Float16 *Vth = nullptr, *Vtl = nullptr;
  BatchScalars S{};
  std::vector<BatchInst> inst_h;
  std::vector<int64_t> kpart_off;
  double product_ms = 0.0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* ws64 = nullptr;  // FP64 true-residual workspace (largest problem)
  size_t ws64_bytes = 0;
};

namespace {

template <typename T> hipError_t plan_alloc(krr_batch_plan* P, T** out, int64_t count) {
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  P->allocs.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return hipSuccess;
}

template <typename T> hipError_t upload(T* dst, const std::vector<T>& src, hipStream_t st) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// Work items of the batched product for a granularity of g column tiles per item; updates
// nsplit / partial offsets in meta_h and inst_h. Items are sorted by cost, largest first.
std::vector<BatchItem> build_items(krr_batch_plan* P, int g) {
  std::vector<BatchItem> items;
  std::vector<std::pair<int64_t, BatchItem>> keyed;
  int64_t off = 0;
  for (int i = 0; i < P->count; ++i) {
    const int64_t n = P->probs[i].n;
    const int64_t rows_pad = round_up(n, ROW_PAD);
    const int64_t tiles = ceil_div(n, 64);
    const int nsplit = (int)ceil_div(tiles, g);
    BatchMeta& M = P->meta_h[i];
    BatchInst& I = P->inst_h[i];
    M.nsplit = nsplit;
    M.part = P->kpart + off;
    M.part_stride = rows_pad * P->M;
    I.part = M.part;
    I.part_stride = M.part_stride;
    off += (int64_t)nsplit * rows_pad * P->M;
    for (int64_t rb = 0; rb < ceil_div(n, 128); ++rb)
      for (int sp = 0; sp < nsplit; ++sp) {
        const int64_t nt = std::min<int64_t>(g, tiles - (int64_t)sp * g);
        BatchItem it{i, g, rb, sp};
        keyed.push_back({nt * I.Kp, it});
      }
  }
  std::stable_sort(keyed.begin(), keyed.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  for (auto& k : keyed) items.push_back(k.second);
  return items;
}

int64_t kpart_elems(krr_batch_plan* P, int g) {
  int64_t tot = 0;
  for (int i = 0; i < P->count; ++i) {
    const int64_t n = P->probs[i].n;
    tot += ceil_div(ceil_div(n, 64), g) * round_up(n, ROW_PAD) * P->M;
  }
  return tot;
}

hipError_t batch_product(krr_batch_plan* P, hipStream_t st) {
  hipError_t e = batch_split_v(P->row_inst, P->meta, P->S.live, P->count, P->N, P->M, P->pf,
                               P->red, P->nred, P->colmax, P->Vth, P->Vtl, P->vscale,
                               P->M <= 8, st);
  if (e != hipSuccess) return e;
  e = batch_compact_live(P->items, P->nitems, P->S.live, P->chunk_cnt, P->live_list,
                         P->live_count, st);
  if (e != hipSuccess) return e;
  e = matmat_batch(P->items, P->live_list, P->live_count, P->inst, P->counter, P->M <= 8, P->grid,
                   st);
  if (e != hipSuccess) return e;
  return batch_finalize(P->meta, P->row_inst, P->S.live, P->N, P->M, P->pf, P->q, st);
}

// One PCG iteration for every problem (the captured graph body).
hipError_t batch_iteration(krr_batch_plan* P, hipStream_t st) {
  const int M = P->M;
  hipError_t e;
  if ((e = batch_product(P, st))) return e;
  if ((e = batch_dot<float, double>(P->pf, P->q, M, P->red, P->nred, P->S.live, P->part_pq, st))) return e;
  if ((e = batch_alpha(P->meta, P->count, M, P->part_pq, P->S, st))) return e;
  if ((e = batch_update_xr(P->row_inst, P->N, M, P->S.alpha, P->pf, P->q, P->x, P->r, st))) return e;
  if ((e = batch_dot<double, double>(P->r, P->r, M, P->red, P->nred, P->S.live, P->part_rr, st))) return e;
  if ((e = batch_conv(P->meta, P->count, M, P->part_rr, P->S, st))) return e;
  if ((e = batch_precond(P->meta, P->count, P->pitems, P->npitems, P->zitems, P->nzitems, P->smax,
                         P->S.live, P->r, M, P->pc_part, P->T, P->z, st)))
    return e;
  if ((e = batch_dot<double, double>(P->r, P->z, M, P->red, P->nred, P->S.live, P->part_rz, st))) return e;
  if ((e = batch_beta(P->meta, P->count, M, P->part_rz, P->part_rr, P->S, st))) return e;
  return batch_update_p(P->row_inst, P->N, M, P->S.beta, P->S.active, 0, P->z, P->p, P->pf, st);
}

// FP64 true-residual scratch of one problem of a batch
struct BatchResid {
  MatmatCtx c;
  double *ax, *res, *prr, *pyy;
};
void layout_batch_resid(Bump& b, BatchResid& R, int64_t n, int64_t d, int64_t m) {
  layout_matmat(b, R.c, n, n, d, m, KRR_PREC_FP64, true, true);
  R.ax = b.take<double>(n * m);
  R.res = b.take<double>(n * m);
  R.prr = b.take<double>(NBLK * m);
  R.pyy = b.take<double>(NBLK * m);
}

// Per-column ||Y - (K + lambda I) alpha|| / ||Y|| of one problem, all in FP64.
krr_status batch_true_residual(krr_batch_plan* P, const krr_batch_problem& b, double* rel,
                               hipStream_t st, double* r_out = nullptr, int64_t ldr = 0) {
  Bump bb(P->ws64);
  BatchResid R;
  layout_batch_resid(bb, R, b.n, b.d, b.m);
  const int64_t n = b.n, m = b.m;
  CHECK_HIP(prepare_points(R.c, b.X, b.ldx, nullptr, 0, b.sigma, st));
  CHECK_HIP(run_matmat(R.c, nullptr, b.alpha, b.lda, false, st));
  CHECK_HIP(matmat_finalize<double>(R.c.part, R.c.part_stride, R.c.nsplit, n, m, m, b.lambda,
                                    b.alpha, b.lda, R.ax, m, st));
  CHECK_HIP(residual_from(b.Y, b.ldy, R.ax, n, m, R.res, st));
  if (r_out) CHECK_HIP(copy2d(R.res, m, r_out, ldr, n, m, st));
  CHECK_HIP(dot_partial<double, double>(R.res, m, R.res, m, n, m, R.prr, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(b.Y, b.ldy, b.Y, b.ldy, n, m, R.pyy, NBLK, st));
  std::vector<double> prr(NBLK * m), pyy(NBLK * m);
  CHECK_HIP(hipMemcpyAsync(prr.data(), R.prr, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipMemcpyAsync(pyy.data(), R.pyy, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  for (int64_t c = 0; c < m; ++c) {
    double rr = 0.0, yy = 0.0;
    for (int k = 0; k < NBLK; ++k) { rr += prr[k * m + c]; yy += pyy[k * m + c]; }
    rel[c] = yy > 0.0 ? std::sqrt(rr / yy) : std::sqrt(rr);
  }
  return KRR_OK;
}

void plan_free(krr_batch_plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  for (void* a : P->allocs) (void)hipFree(a);
  delete P;
}

}  // namespace

extern "C" {

krr_status krr_batch_plan_create(const krr_batch_problem* probs, int32_t count,
                                 const krr_pcg_opts* opts, krr_batch_plan** plan_out,
                                 void* stream) {
  g_err[0] = 0;
  if (!probs || count < 1 || !plan_out) return fail(KRR_E_ARG, "krr_batch_plan_create: bad arguments");
  *plan_out = nullptr;
  krr_pcg_opts o;
  krr_pcg_defaults(&o);
  if (opts) o = *opts;
  if (o.prec != KRR_PREC_F16X3)
    return fail(KRR_E_ARG, "krr_batch_plan_create: batched products use KRR_PREC_F16X3");
  if (!(o.tol > 0.0) || o.max_iter < 1) return fail(KRR_E_ARG, "krr_batch_plan_create: bad tol/max_iter");
  if (o.check_every < 1) o.check_every = 1;
  if (o.check_every > KRR_BATCH_MAX_GROUP) o.check_every = KRR_BATCH_MAX_GROUP;
  int M = 0;
  for (int i = 0; i < count; ++i) {
    const krr_batch_problem& b = probs[i];
    if (!b.X || !b.Y || !b.alpha || b.n < 2 || b.d < 1 || b.ldx < b.d || b.m < 1 ||
        b.m > KRR_BATCH_MAX_M || b.ldy < b.m || b.lda < b.m)
      return fail(KRR_E_ARG, "krr_batch_plan_create: problem %d: bad pointer or size", i);
    if (!(b.sigma > 0.0) || !(b.lambda > 0.0) || !std::isfinite(b.sigma) || !std::isfinite(b.lambda))
      return fail(KRR_E_ARG, "krr_batch_plan_create: problem %d: sigma and lambda must be > 0", i);
    if (b.Ut && (b.s < 1 || b.s >= b.n || b.ldu < b.s))
      return fail(KRR_E_ARG, "krr_batch_plan_create: problem %d: need 1 <= s < n", i);
    M = std::max<int>(M, (int)b.m);
  }
  hipStream_t st = (hipStream_t)stream;
  krr_batch_plan* P = new krr_batch_plan();
  P->count = count;
  P->M = M;
  P->opts = o;
  P->probs.assign(probs, probs + count);
  P->meta_h.resize(count);
  P->inst_h.resize(count);
  auto bail = [&](krr_status code) { plan_free(P); return code; };
#define PLAN_HIP(...)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (__VA_ARGS__);                                                           \
    if (e_ != hipSuccess) {                                                                  \
      fail(KRR_E_HIP, "%s failed: %s (line %d)", #__VA_ARGS__, hipGetErrorString(e_), __LINE__); \
      return bail(KRR_E_HIP);                                                                \
    }                                                                                        \
  } while (0)

  // packed layout and per-problem metadata
  std::vector<int> row_inst_h;
  std::vector<RedItem> red_h;
  std::vector<PCItem> pitems_h;
  std::vector<ZItem> zitems_h;
  int64_t off = 0, pc_off = 0, t_off = 0, nmax = 0;
  for (int i = 0; i < count; ++i) {
    const krr_batch_problem& b = probs[i];
    BatchMeta& Mt = P->meta_h[i];
    const int64_t rows_pad = round_up(b.n, ROW_PAD);
    Mt.off = off;
    Mt.n = b.n;
    Mt.m = (int)b.m;
    Mt.lambda = b.lambda;
    Mt.has_u = (b.Ut && o.use_precond) ? 1 : 0;
    Mt.Ut = b.Ut;
    Mt.s = Mt.has_u ? b.s : 0;
    Mt.ldu = b.ldu;
    Mt.inv_lp = 1.0 / (b.lambda_p > 0.0 ? b.lambda_p : b.lambda);
    Mt.ext_in = b.Y;
    Mt.ld_in = b.ldy;
    Mt.ext_out = b.alpha;
    Mt.ld_out = b.lda;
    Mt.red_begin = (int)red_h.size();
    for (int64_t r0 = 0; r0 < b.n; r0 += 1024)
      red_h.push_back(RedItem{i, off + r0, off + std::min<int64_t>(b.n, r0 + 1024)});
    Mt.red_end = (int)red_h.size();
    if (Mt.has_u) {
      const int chunks = (int)std::max<int64_t>(1, ceil_div(b.n, 512));  // rows per first-pass item
      Mt.pc_chunks = chunks;
      Mt.pc_part_off = pc_off;
      Mt.t_off = t_off;
      const int64_t rpc = ceil_div(b.n, chunks);
      for (int64_t k0 = 0; k0 < b.s; k0 += 256)
        for (int c = 0; c < chunks; ++c)
          pitems_h.push_back(PCItem{i, c, k0, c * rpc, std::min<int64_t>(b.n, (c + 1) * rpc), pc_off});
      pc_off += (int64_t)chunks * b.s * 16;
      t_off += b.s * 16;
      P->smax = std::max<int64_t>(P->smax, b.s);
    }
    for (int64_t i0 = 0; i0 < b.n; i0 += 64) zitems_h.push_back(ZItem{i, i0});
    for (int64_t r = 0; r < rows_pad; ++r) row_inst_h.push_back(i);
    off += rows_pad;
    nmax = std::max<int64_t>(nmax, b.n);
  }
  P->N = off;
  P->nred = (int)red_h.size();
  P->npitems = (int)pitems_h.size();
  P->nzitems = (int)zitems_h.size();
  const int64_t NM = P->N * M;
  PLAN_HIP(plan_alloc(P, &P->meta, count));
  PLAN_HIP(plan_alloc(P, &P->row_inst, P->N));
  PLAN_HIP(plan_alloc(P, &P->inst, count));
  PLAN_HIP(plan_alloc(P, &P->counter, 64));
  PLAN_HIP(plan_alloc(P, &P->red, P->nred));
  PLAN_HIP(plan_alloc(P, &P->pitems, P->npitems));
  PLAN_HIP(plan_alloc(P, &P->zitems, P->nzitems));
  PLAN_HIP(plan_alloc(P, &P->pf, NM));
  PLAN_HIP(plan_alloc(P, &P->x, NM));
  PLAN_HIP(plan_alloc(P, &P->r, NM));
  PLAN_HIP(plan_alloc(P, &P->z, NM));
  PLAN_HIP(plan_alloc(P, &P->p, NM));
  PLAN_HIP(plan_alloc(P, &P->q, NM));
  PLAN_HIP(plan_alloc(P, &P->part_yy, (int64_t)P->nred * M));
  PLAN_HIP(plan_alloc(P, &P->part_rr, (int64_t)P->nred * M));
  PLAN_HIP(plan_alloc(P, &P->part_pq, (int64_t)P->nred * M));
  PLAN_HIP(plan_alloc(P, &P->part_rz, (int64_t)P->nred * M));
  PLAN_HIP(plan_alloc(P, &P->pc_part, pc_off));
  PLAN_HIP(plan_alloc(P, &P->T, t_off));
  PLAN_HIP(plan_alloc(P, &P->colmax, (int64_t)count * 16));
  PLAN_HIP(plan_alloc(P, &P->vscale, (int64_t)count * 16));
  PLAN_HIP(plan_alloc(P, &P->Vth, 16 * P->N));
  PLAN_HIP(plan_alloc(P, &P->Vtl, 16 * P->N));
  const int cm = count * M;
  PLAN_HIP(plan_alloc(P, &P->S.ynorm, cm));
  PLAN_HIP(plan_alloc(P, &P->S.rnorm, cm));
  PLAN_HIP(plan_alloc(P, &P->S.rho, cm));
  PLAN_HIP(plan_alloc(P, &P->S.alpha, cm));
  PLAN_HIP(plan_alloc(P, &P->S.beta, cm));
  PLAN_HIP(plan_alloc(P, &P->S.active, cm));
  PLAN_HIP(plan_alloc(P, &P->S.broken, cm));
  PLAN_HIP(plan_alloc(P, &P->S.col_iters, cm));
  PLAN_HIP(plan_alloc(P, &P->S.count, 64));
  PLAN_HIP(plan_alloc(P, &P->S.iter, 64));
  PLAN_HIP(plan_alloc(P, &P->S.live, count));
  PLAN_HIP(fill_i32(P->S.live, count, 1, st));
  PLAN_HIP(plan_alloc(P, &P->S.tol, cm));
  // per-problem prepared points (F16X3, scaled). Up to d = 128 the norm terms of the
  // exponent are added in the epilogue of the register-resident body, so the operands hold
  // only the coordinates (width round_up(d, 32), the same array on both sides); larger d
  // keeps the two augmented norm columns for the large-d body.
  for (int i = 0; i < count; ++i) {
    const krr_batch_problem& b = probs[i];
    const int64_t rows_pad = round_up(b.n, ROW_PAD);
    const bool ne = round_up(b.d, K_STEP) <= 128;
    const int64_t Kp = ne ? round_up(b.d, K_STEP) : kp_for(b.d);
    _Float16 *ah, *al, *bh = nullptr, *bl = nullptr;
    float *stats, *nrm = nullptr;
    PLAN_HIP(plan_alloc(P, &ah, rows_pad * Kp));
    PLAN_HIP(plan_alloc(P, &al, rows_pad * Kp));
    if (ne) {
      PLAN_HIP(plan_alloc(P, &nrm, rows_pad));
    } else {
      PLAN_HIP(plan_alloc(P, &bh, rows_pad * Kp));
      PLAN_HIP(plan_alloc(P, &bl, rows_pad * Kp));
    }
    PLAN_HIP(plan_alloc(P, &stats, 64));
    const double c2 = 1.4426950408889634 / (2.0 * b.sigma * b.sigma);
    PLAN_HIP(fill_f32(stats, 4, 0.0f, st));
    PLAN_HIP(point_stats(b.X, b.n, b.d, b.ldx, stats, st));
    RowSpec rs;
    rs.c2 = c2;
    PLAN_HIP(prep_points<_Float16>(b.X, b.n, b.d, b.ldx, rows_pad, Kp, rs, stats, 0, 0, ah, al,
                                   stats + 2, st, nrm));
    if (!ne)
      PLAN_HIP(prep_points<_Float16>(b.X, b.n, b.d, b.ldx, rows_pad, Kp, rs, stats, 1, 0, bh, bl,
                                     nullptr, st));
    BatchInst& I = P->inst_h[i];
    I.Ahi = ah; I.Alo = al;
    I.Bhi = ne ? ah : bh;
    I.Blo = ne ? al : bl;
    I.nrm = nrm;
    I.Vth = P->Vth + P->meta_h[i].off;
    I.Vtl = P->Vtl + P->meta_h[i].off;
    I.vscale = P->vscale + 16 * i;
    I.qinv2 = stats + 2;
    I.n = b.n;
    I.m = M;
    I.ldvt = P->N;
    I.ldp = M;
    I.Kp = (int)Kp;
  }
  // product partials sized for the finest candidate granularity
  const int cands[4] = {4, 8, 16, 32};
  PLAN_HIP(plan_alloc(P, &P->kpart, kpart_elems(P, cands[0])));
  PLAN_HIP(upload(P->row_inst, row_inst_h, st));
  PLAN_HIP(upload(P->red, red_h, st));
  PLAN_HIP(upload(P->pitems, pitems_h, st));
  PLAN_HIP(upload(P->zitems, zitems_h, st));
  PLAN_HIP(fill_f32(P->pf, NM, 0.0f, st));
  for (double* v : {P->x, P->r, P->z, P->p, P->q}) PLAN_HIP(fill_f64(v, NM, 0.0, st));
  int dev = 0, cus = 256;
  PLAN_HIP(hipGetDevice(&dev));
  PLAN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  P->grid = 2 * cus;
  // autotune the work-item granularity on the real problem set (the finest granularity
  // has the most items, so its buffer holds every candidate's list)
  {
    const int64_t maxitems = (int64_t)build_items(P, cands[0]).size();
    PLAN_HIP(plan_alloc(P, &P->items, maxitems));
    PLAN_HIP(plan_alloc(P, &P->live_list, maxitems));
    PLAN_HIP(plan_alloc(P, &P->live_count, 64));
    PLAN_HIP(plan_alloc(P, &P->chunk_cnt, ceil_div(maxitems, 256) + 64));
  }
  hipEvent_t e0, e1;
  PLAN_HIP(hipEventCreate(&e0));
  PLAN_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_g = cands[0];
  for (int g : cands) {
    std::vector<BatchItem> items = build_items(P, g);
    PLAN_HIP(upload(P->items, items, st));
    PLAN_HIP(upload(P->inst, P->inst_h, st));
    PLAN_HIP(upload(P->meta, P->meta_h, st));
    P->nitems = (int)items.size();
    float tbest = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      PLAN_HIP(hipEventRecord(e0, st));
      PLAN_HIP(batch_product(P, st));
      PLAN_HIP(hipEventRecord(e1, st));
      PLAN_HIP(hipEventSynchronize(e1));
      float t = 0.0f;
      PLAN_HIP(hipEventElapsedTime(&t, e0, e1));
      if (rep > 0) tbest = std::min(tbest, t);
    }
    if (tbest < best) {
      best = tbest;
      best_g = g;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::vector<BatchItem> items = build_items(P, best_g);
    PLAN_HIP(upload(P->items, items, st));
    P->nitems = (int)items.size();
    PLAN_HIP(upload(P->inst, P->inst_h, st));
    PLAN_HIP(upload(P->meta, P->meta_h, st));
  }
  P->tiles_per_item = best_g;
  P->product_ms = best;
  // FP64 true-residual workspace (the largest problem)
  if (o.true_residual) {
    for (int i = 0; i < count; ++i) {
      Bump sz(nullptr);
      BatchResid R;
      layout_batch_resid(sz, R, probs[i].n, probs[i].d, probs[i].m);
      P->ws64_bytes = std::max(P->ws64_bytes, sz.off);
    }
    char* w = nullptr;
    PLAN_HIP(plan_alloc(P, &w, (int64_t)P->ws64_bytes));
    P->ws64 = w;
  }
  PLAN_HIP(hipStreamSynchronize(st));
  // capture check_every iterations: one graph launch and one host read of the active count
  // per group
  PLAN_HIP(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
  PLAN_HIP(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
  {
    hipError_t ce = hipSuccess;
    for (int k = 0; k < o.check_every && ce == hipSuccess; ++k) ce = batch_iteration(P, P->cap);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(P->cap, &g);
    P->graph = g;
    PLAN_HIP(ce);
    PLAN_HIP(ee);
  }
  PLAN_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
#undef PLAN_HIP
  *plan_out = P;
  return KRR_OK;
}

void krr_batch_plan_destroy(krr_batch_plan* plan) { plan_free(plan); }

// PCG on the packed right-hand sides in P->r (x from zero) with per-column tolerances
// already in S.tol; returns the iterations run.
static krr_status batch_pcg(krr_batch_plan* P, int* iters, double* ms, hipStream_t st) {
  const int M = P->M;
  CHECK_HIP(fill_f64(P->x, P->N * M, 0.0, st));
  CHECK_HIP(fill_i32(P->S.live, P->count, 1, st));  // start-up reductions cover every problem
  CHECK_HIP(batch_dot<double, double>(P->r, P->r, M, P->red, P->nred, P->S.live, P->part_yy, st));
  CHECK_HIP(batch_precond(P->meta, P->count, P->pitems, P->npitems, P->zitems, P->nzitems, P->smax,
                          P->S.live, P->r, M, P->pc_part, P->T, P->z, st));
  CHECK_HIP(batch_dot<double, double>(P->r, P->z, M, P->red, P->nred, P->S.live, P->part_rz, st));
  CHECK_HIP(batch_init_scalars(P->meta, P->count, M, P->part_yy, P->part_rz, P->S, st));
  CHECK_HIP(batch_update_p(P->row_inst, P->N, M, P->S.beta, P->S.active, 1, P->z, P->p, P->pf, st));
  int h_count = 0;
  CHECK_HIP(hipMemcpyAsync(&h_count, P->S.count, sizeof(int), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  hipEvent_t e0, e1;
  CHECK_HIP(hipEventCreate(&e0));
  CHECK_HIP(hipEventCreate(&e1));
  int it = 0;
  hipError_t err = hipEventRecord(e0, st);
  while (err == hipSuccess && h_count > 0 && it < P->opts.max_iter) {
    err = hipGraphLaunch(P->exec, st);  // check_every iterations
    it += P->opts.check_every;
    if (err == hipSuccess) {
      err = hipMemcpyAsync(&h_count, P->S.count, sizeof(int), hipMemcpyDeviceToHost, st);
      if (err == hipSuccess) err = hipStreamSynchronize(st);
    }
  }
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.0f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  CHECK_HIP(err);
  *iters = it;
  *ms = t;
  return KRR_OK;
}

krr_status krr_batch_solve(krr_batch_plan* P, krr_batch_report* rep, void* stream) {
  g_err[0] = 0;
  if (!P) return fail(KRR_E_ARG, "krr_batch_solve: NULL plan");
  hipStream_t st = (hipStream_t)stream;
  const int M = P->M, cm = P->count * M;
  const double tol = P->opts.tol;
  std::vector<double> tolv(cm, 1.0);
  for (int i = 0; i < P->count; ++i)
    for (int c = 0; c < P->probs[i].m; ++c) tolv[i * M + c] = tol;
  CHECK_HIP(hipMemcpyAsync(P->S.tol, tolv.data(), sizeof(double) * cm, hipMemcpyHostToDevice, st));
  CHECK_HIP(batch_pack(P->row_inst, P->meta, P->N, M, BATCH_PACK_IN, P->r, st));
  int it = 0;
  double ms = 0.0;
  CHECK_ST(batch_pcg(P, &it, &ms, st));
  CHECK_HIP(batch_pack(P->row_inst, P->meta, P->N, M, BATCH_UNPACK_SET, P->x, st));
  int total_iters = it;
  const double iter_ms = it > 0 ? ms / it : 0.0;
  std::vector<double> rn(cm), yn(cm);
  std::vector<int> brk(cm), cit(cm);
  CHECK_HIP(hipMemcpyAsync(cit.data(), P->S.col_iters, sizeof(int) * cm, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipMemcpyAsync(rn.data(), P->S.rnorm, sizeof(double) * cm, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipMemcpyAsync(yn.data(), P->S.ynorm, sizeof(double) * cm, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipMemcpyAsync(brk.data(), P->S.broken, sizeof(int) * cm, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  int conv = 0, nbrk = 0;
  for (int i = 0; i < P->count; ++i)
    for (int c = 0; c < P->probs[i].m; ++c) {
      const int e = i * M + c;
      const double rel = yn[e] > 0.0 ? rn[e] / yn[e] : 0.0;
      if (brk[e]) ++nbrk;
      else if (rel <= tol) ++conv;
      if (rep && rep->relres_rec) rep->relres_rec[i * KRR_BATCH_MAX_M + c] = rel;
      if (rep && rep->col_iters) rep->col_iters[i * KRR_BATCH_MAX_M + c] = cit[e];
    }
  // FP64 true residuals; refinement solves A delta = R for the columns above tol
  std::vector<double> rel_true(cm, 0.0);
  int refine_steps = 0;
  const bool want_true = P->opts.true_residual || P->opts.refine > 0;
  auto true_all = [&]() -> krr_status {
    for (int i = 0; i < P->count; ++i) {
      // R also lands in the packed right-hand side, ready for a refinement solve
      const krr_status stt = batch_true_residual(P, P->probs[i], &rel_true[i * M], st,
                                                 P->r + P->meta_h[i].off * M, M);
      if (stt != KRR_OK) return stt;
    }
    return KRR_OK;
  };
  if (want_true && nbrk == 0) {
    CHECK_ST(true_all());
    while (refine_steps < P->opts.refine) {
      double worst = 0.0;
      for (int i = 0; i < P->count; ++i)
        for (int c = 0; c < P->probs[i].m; ++c) worst = std::max(worst, rel_true[i * M + c]);
      if (!(worst > tol)) break;
      ++refine_steps;
      // P->r holds every problem's R; settled columns stay inactive
      for (int i = 0; i < P->count; ++i) {
        const krr_batch_problem& b = P->probs[i];
        for (int c = 0; c < M; ++c) {
          const double r = c < b.m ? rel_true[i * M + c] : 0.0;
          tolv[i * M + c] = r > tol ? std::max(0.5 * tol / r, 1e-14) : 1.0;
        }
      }
      CHECK_HIP(hipMemcpyAsync(P->S.tol, tolv.data(), sizeof(double) * cm, hipMemcpyHostToDevice, st));
      int it2 = 0;
      double ms2 = 0.0;
      CHECK_ST(batch_pcg(P, &it2, &ms2, st));
      total_iters += it2;
      CHECK_HIP(batch_pack(P->row_inst, P->meta, P->N, M, BATCH_UNPACK_ADD, P->x, st));
      CHECK_ST(true_all());
    }
  }
  if (rep && rep->relres_true)
    for (int i = 0; i < P->count; ++i)
      for (int c = 0; c < P->probs[i].m; ++c)
        rep->relres_true[i * KRR_BATCH_MAX_M + c] = want_true && nbrk == 0 ? rel_true[i * M + c] : NAN;
  if (rep) {
    rep->iters = total_iters;
    rep->converged_cols = conv;
    rep->breakdown_cols = nbrk;
    rep->refine_steps = refine_steps;
    rep->product_ms = P->product_ms;
    rep->iteration_ms = iter_ms;
    rep->tiles_per_item = P->tiles_per_item;
    rep->work_items = P->nitems;
  }
  if (nbrk > 0) return fail(KRR_E_BREAKDOWN, "krr_batch_solve: %d column(s) broke down", nbrk);
  bool ok = true;
  if (refine_steps > 0) {
    for (int i = 0; i < P->count; ++i)
      for (int c = 0; c < P->probs[i].m; ++c) ok = ok && rel_true[i * M + c] <= tol;
  } else {
    int total = 0;
    for (int i = 0; i < P->count; ++i) total += (int)P->probs[i].m;
    ok = conv == total;
  }
  if (!ok)
    return fail(KRR_E_NO_CONV, "krr_batch_solve: not converged after %d iterations", total_iters);
  return KRR_OK;
}

}  // extern "C"
