// C ABI of the learned-preconditioner kernels (include/mfmlp.h).
#include <cstdint>

#include "mf_internal.h"
#include "mfcheb.h"
#include "mfmlp.h"

namespace mf {

static bool aligned16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

}  // namespace mf

using namespace mf;

extern "C" {

int mf_mlp_gemm(int M, int N, int K, int ta, int tb, const uint16_t* A, int64_t lda,
                const uint16_t* B, int64_t ldb, int kchunk, const float* bias, int relu,
                const uint16_t* mask, int64_t ldmask, float* out_f32, int64_t ld_f32, int atomic,
                uint16_t* out_bf16, int64_t ld_bf16, int kb, void* stream) {
  if (!A || !B) return fail(MF_ERR_ARG, "A and B must be non-NULL");
  if (!out_f32 && !out_bf16) return fail(MF_ERR_ARG, "no output");
  if (M < 1 || N < 1 || K < 1 || M % 8 || N % 8 || K % 8)
    return fail(MF_ERR_ARG, "M, N, K must be positive multiples of 8");
  if (lda % 8 || ldb % 8 || !aligned16(A) || !aligned16(B))
    return fail(MF_ERR_ARG, "lda, ldb must be multiples of 8 and A, B 16-byte aligned");
  if (kb < 0 || kb % 8) return fail(MF_ERR_ARG, "kb must be 0 or a positive multiple of 8");
  if (kb > 0) {  // cell-blocked B and outputs: N in blocks of kb, block strides ldb, ld_f32, ld_bf16
    if (tb || mask) return fail(MF_ERR_ARG, "the blocked layout takes neither tb nor a mask");
    if (N % kb) return fail(MF_ERR_ARG, "N must be a multiple of kb");
    if (lda < (ta ? M : K) || ldb < (int64_t)K * kb || (out_f32 && ld_f32 < (int64_t)M * kb) ||
        (out_bf16 && ld_bf16 < (int64_t)M * kb))
      return fail(MF_ERR_ARG, "block stride below (rows of the block) x kb");
  } else {
    if (lda < (ta ? M : K) || ldb < (tb ? K : N))
      return fail(MF_ERR_ARG, "leading dimension too small");
    if ((out_f32 && ld_f32 < N) || (out_bf16 && ld_bf16 < N) || (mask && ldmask < N))
      return fail(MF_ERR_ARG, "output leading dimension < N");
  }
  if (atomic && !out_f32) return fail(MF_ERR_ARG, "atomic needs out_f32");
  if (kchunk > 0 && (bias || relu || mask || out_bf16 || !atomic))
    return fail(MF_ERR_ARG, "a split K range needs atomic FP32 output without epilogue ops");
  GemmEpi ep{bias, relu, mask, ldmask, out_f32, ld_f32, atomic, out_bf16, ld_bf16, kb};
  hipError_t err = launch_gemm_bf16(M, N, K, ta != 0, tb != 0, A, lda, B, ldb, kchunk, ep,
                                    static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "MLP GEMM launch");
  return MF_OK;
}

int mf_cell_gather(mf_operator* handle, int k, const double* R, int64_t ldr, const double* E,
                   int64_t lde, int Fp, uint16_t* X0t, float* Tt, int64_t ldx, float* rho,
                   int pou_sqrt, const double* dscale, int blocked, void* stream) {
  if (!handle || !R || !X0t) return fail(MF_ERR_ARG, "operator, R, X0t non-NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (op->refined) return fail(MF_ERR_UNSUPPORTED, "cell gather/scatter are built for uniform box meshes");
  const int F = op->np * op->np * op->np;
  if (k < 1 || ldr < k || (E && lde < k)) return fail(MF_ERR_ARG, "need k >= 1, ld >= k");
  if (E && !Tt) return fail(MF_ERR_ARG, "E needs Tt");
  if (Fp < F || Fp % 8) return fail(MF_ERR_ARG, "Fp must be >= np^3 and a multiple of 8");
  if (!blocked && ldx < op->ncells * k) return fail(MF_ERR_ARG, "ldx < ncells * k");
  if (blocked && ldx < (int64_t)Fp * k) return fail(MF_ERR_ARG, "blocked: ldx < Fp * k");
  if (op->ncells * k >= ((int64_t)1 << 31)) return fail(MF_ERR_UNSUPPORTED, "batch too large");
  hipError_t err = launch_cell_gather(*op, k, R, ldr, E, lde, Fp, X0t, Tt, ldx, rho, pou_sqrt,
                                      dscale, blocked, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "cell gather launch");
  return MF_OK;
}

int mf_cell_scatter(mf_operator* handle, int k, const float* Yt, int64_t ldy, const float* rho,
                    const double* diag, const double* R, int64_t ldr, double* Z, int64_t ldz,
                    int pou_sqrt, const double* dscale, int blocked, void* stream) {
  if (!handle || !Yt || !Z) return fail(MF_ERR_ARG, "operator, Yt, Z non-NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (op->refined) return fail(MF_ERR_UNSUPPORTED, "cell gather/scatter are built for uniform box meshes");
  if (k < 1 || ldz < k) return fail(MF_ERR_ARG, "need k >= 1, ldz >= k");
  const int F = op->np * op->np * op->np;
  if (!blocked && ldy < op->ncells * k) return fail(MF_ERR_ARG, "ldy < ncells * k");
  if (blocked && ldy < (int64_t)F * k) return fail(MF_ERR_ARG, "blocked: ldy < np^3 * k");
  if (diag && (!R || ldr < k)) return fail(MF_ERR_ARG, "diag needs R with ldr >= k");
  if (R && R == Z) return fail(MF_ERR_ARG, "Z must not be R");
  hipError_t err = launch_cell_scatter(*op, k, Yt, ldy, rho, diag, R, ldr, Z, ldz, pou_sqrt,
                                       dscale, blocked, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "cell scatter launch");
  return MF_OK;
}

int64_t mf_skip_floor_work(int F) {
  const int64_t eig = mf_sym_eig_work(F);
  if (eig < 0) return -1;
  return 2 * (int64_t)F * F + ((F + 7) / 8) * 8 + eig;
}

int mf_skip_floor(int F, float* S, int64_t lds, uint16_t* Sbf, int64_t ldsb, double margin,
                  double* work, int64_t work_len, int* status, void* stream) {
  if (!(margin >= 0.0)) return fail(MF_ERR_ARG, "margin must be >= 0");
  if (!S || !Sbf || !work || !status) return fail(MF_ERR_ARG, "S, Sbf, work, status non-NULL");
  const int64_t need = mf_skip_floor_work(F);
  if (need < 0) return fail(MF_ERR_UNSUPPORTED, "need 1 <= F <= 2048");
  if (lds < F || ldsb < F) return fail(MF_ERR_ARG, "need lds, ldsb >= F");
  if (work_len < need) return fail(MF_ERR_ARG, "work shorter than mf_skip_floor_work(F)");
  double* A = work;                        // F x F, the symmetrised block
  double* V = A + (int64_t)F * F;          // F x F, eigenvectors
  double* w = V + (int64_t)F * F;          // F eigenvalues (padded to 8)
  double* ew = w + ((F + 7) / 8) * 8;      // mf_sym_eig's own work
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t err = launch_skip_sym(F, S, lds, A, s);
  if (err != hipSuccess) return hip_fail(err, "skip symmetrise launch");
  if (int st = mf_sym_eig(F, A, F, w, V, F, 0.0, status, ew, need - (ew - work), stream)) return st;
  err = launch_skip_rebuild(F, V, w, margin, S, lds, Sbf, ldsb, s);
  if (err != hipSuccess) return hip_fail(err, "skip rebuild launch");
  return MF_OK;
}

int mf_mse_grad(int F, int Fp, int64_t N, const float* Yt, const float* Tt, int64_t ld,
                const float* roww, float scale, uint16_t* dYt, double* loss, void* stream) {
  if (!Yt || !Tt || !dYt || !loss) return fail(MF_ERR_ARG, "NULL argument");
  if (F < 1 || Fp < F || N < 1 || ld < N) return fail(MF_ERR_ARG, "need 1 <= F <= Fp, 1 <= N <= ld");
  hipError_t err = launch_mse_grad(F, Fp, N, Yt, Tt, ld, roww, scale, dYt, loss,
                                   static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "MSE kernel launch");
  return MF_OK;
}

int mf_row_sums(int M, int64_t N, const uint16_t* X, int64_t ld, float* out, int accumulate,
                void* stream) {
  if (!X || !out) return fail(MF_ERR_ARG, "NULL argument");
  if (M < 1 || N < 1 || ld < N) return fail(MF_ERR_ARG, "need M, N >= 1, ld >= N");
  hipError_t err = launch_row_sums(M, N, X, ld, out, accumulate != 0, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "row-sum kernel launch");
  return MF_OK;
}

int mf_adam(int64_t n, float* w, const float* g, float* m1, float* m2, uint16_t* wbf, float lr,
            float beta1, float beta2, float eps, int step, void* stream) {
  if (!w || !g || !m1 || !m2) return fail(MF_ERR_ARG, "NULL argument");
  if (n < 1 || step < 1) return fail(MF_ERR_ARG, "need n >= 1, step >= 1");
  hipError_t err = launch_adam(n, w, g, m1, m2, wbf, lr, beta1, beta2, eps, step,
                               static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "Adam kernel launch");
  return MF_OK;
}

int mf_symmetrize(int n, float* S, int64_t ld, uint16_t* Sbf, void* stream) {
  if (!S || n < 1 || ld < n) return fail(MF_ERR_ARG, "need S non-NULL, n >= 1, ld >= n");
  hipError_t err = launch_symmetrize(n, S, ld, Sbf, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "symmetrize kernel launch");
  return MF_OK;
}

int mf_to_bf16(int64_t n, const float* src, uint16_t* dst, void* stream) {
  if (!src || !dst || n < 0) return fail(MF_ERR_ARG, "bad arguments");
  if (n == 0) return MF_OK;
  hipError_t err = launch_to_bf16(n, src, dst, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "conversion kernel launch");
  return MF_OK;
}

int mf_fill_f32(int64_t n, float* v, float x, void* stream) {
  if (!v || n < 0) return fail(MF_ERR_ARG, "bad arguments");
  if (n == 0) return MF_OK;
  hipError_t err = launch_fill_f32(v, n, x, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "fill kernel launch");
  return MF_OK;
}

}  // extern "C"
