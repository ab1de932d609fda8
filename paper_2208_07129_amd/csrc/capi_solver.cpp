// C ABI of the block-CG building blocks (include/mfsolve.h).  Gram blocks and
// block updates are the library's FP64 matrix-core kernels (blas64.hip); the
// reductions and the rest are the kernels of solver.hip.
#include <vector>

#include "mf_internal.h"
#include "mfsolve.h"

namespace mf {

static bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* a0 = static_cast<const char*>(a);
  const char* b0 = static_cast<const char*>(b);
  return a0 < b0 + bn && b0 < a0 + an;
}

static size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  return rows > 0 ? (size_t)((rows - 1) * ld + cols) * sizeof(double) : 0;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_diagonal(mf_operator* handle, double* diag, void* stream) {
  if (!handle || !diag) return fail(MF_ERR_ARG, "operator and diag must be non-NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (op->refined) return fail(MF_ERR_UNSUPPORTED, "mf_diagonal is built for uniform box meshes");
  hipError_t err = launch_diagonal(*op, op->d_dtab, diag, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "diagonal kernel launch");
  return MF_OK;
}

int64_t mf_block_gram_work(int64_t n, int k) {
  if (n < 0 || k < 1) return -1;
  return gram_blocks(n) * (int64_t)k * k;
}

int mf_block_gram(int64_t n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double alpha, double beta, double* C, int ldc, double* work, int64_t work_len,
                  void* stream) {
  if (!C || !work || (n > 0 && (!A || !B)))
    return fail(MF_ERR_ARG, "A, B, C and work must be non-NULL");
  if (n < 0 || k < 1 || lda < k || ldb < k || ldc < k)
    return fail(MF_ERR_ARG, "need n >= 0, k >= 1, lda, ldb, ldc >= k");
  if (work_len < mf_block_gram_work(n, k)) return fail(MF_ERR_ARG, "work_len < mf_block_gram_work");
  const size_t cs = span_bytes(k, k, ldc), ws = (size_t)work_len * sizeof(double);
  if (overlaps(C, cs, A, span_bytes(n, k, lda)) || overlaps(C, cs, B, span_bytes(n, k, ldb)) ||
      overlaps(work, ws, C, cs) || overlaps(work, ws, A, span_bytes(n, k, lda)) ||
      overlaps(work, ws, B, span_bytes(n, k, ldb)))
    return fail(MF_ERR_ARG, "C or work overlaps an operand");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  // partial products of row chunks (matrix-core kernel), then their reduction
  const int64_t nb = gram_chunks(n);
  hipError_t err = launch_gram_partial(n, k, A, lda, B, ldb, nb, work, hs);
  if (err == hipSuccess) err = launch_gram_reduce(k, (int)nb, work, alpha, beta, C, ldc, hs);
  if (err != hipSuccess) return hip_fail(err, "Gram kernel launch");
  return MF_OK;
}

int64_t mf_block_gram2_work(int64_t n, int k) {
  if (n < 0 || k < 1) return -1;
  return 2 * gram2_chunks(n) * (int64_t)k * k;
}

int mf_block_gram2(int64_t n, int k, const double* A, int64_t lda, const double* B1, int64_t ldb1,
                   const double* B2, int64_t ldb2, double alpha, double beta, double* C1,
                   int ldc1, double* C2, int ldc2, double* work, int64_t work_len, void* stream) {
  if (!C1 || !C2 || !work || (n > 0 && (!A || !B1 || !B2)))
    return fail(MF_ERR_ARG, "A, B1, B2, C1, C2 and work must be non-NULL");
  if (n < 0 || k < 1 || lda < k || ldb1 < k || ldb2 < k || ldc1 < k || ldc2 < k)
    return fail(MF_ERR_ARG, "need n >= 0, k >= 1, lda, ldb1, ldb2, ldc1, ldc2 >= k");
  if (work_len < mf_block_gram2_work(n, k))
    return fail(MF_ERR_ARG, "work_len < mf_block_gram2_work");
  const size_t c1s = span_bytes(k, k, ldc1), c2s = span_bytes(k, k, ldc2);
  const size_t ws = (size_t)work_len * sizeof(double);
  const size_t as = span_bytes(n, k, lda), b1s = span_bytes(n, k, ldb1), b2s = span_bytes(n, k, ldb2);
  if (overlaps(C1, c1s, C2, c2s) || overlaps(C1, c1s, A, as) || overlaps(C1, c1s, B1, b1s) ||
      overlaps(C1, c1s, B2, b2s) || overlaps(C2, c2s, A, as) || overlaps(C2, c2s, B1, b1s) ||
      overlaps(C2, c2s, B2, b2s) || overlaps(work, ws, C1, c1s) || overlaps(work, ws, C2, c2s) ||
      overlaps(work, ws, A, as) || overlaps(work, ws, B1, b1s) || overlaps(work, ws, B2, b2s))
    return fail(MF_ERR_ARG, "C1, C2 or work overlaps an operand or each other");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int64_t nb = gram2_chunks(n);
  double* work2 = work + nb * (int64_t)k * k;
  hipError_t err = launch_gram2_partial(n, k, A, lda, B1, ldb1, B2, ldb2, nb, work, work2, hs);
  if (err == hipSuccess) err = launch_gram_reduce(k, (int)nb, work, alpha, beta, C1, ldc1, hs);
  if (err == hipSuccess) err = launch_gram_reduce(k, (int)nb, work2, alpha, beta, C2, ldc2, hs);
  if (err != hipSuccess) return hip_fail(err, "Gram kernel launch");
  return MF_OK;
}

int mf_block_update(int64_t n, int k, int kp, double alpha, const double* P, int64_t ldp,
                    const double* M, int ldm, double beta, double* Y, int64_t ldy, void* stream) {
  if (n == 0) return (!M || k < 1 || kp < 1) ? fail(MF_ERR_ARG, "M non-NULL, k, kp >= 1") : MF_OK;
  if (!P || !M || !Y) return fail(MF_ERR_ARG, "P, M and Y must be non-NULL");
  if (n < 0 || k < 1 || kp < 1 || ldp < kp || ldm < k || ldy < k)
    return fail(MF_ERR_ARG, "need n >= 0, k, kp >= 1, ldp >= kp, ldm >= k, ldy >= k");
  const size_t ys = span_bytes(n, k, ldy);
  if (overlaps(Y, ys, P, span_bytes(n, kp, ldp)) || overlaps(Y, ys, M, span_bytes(kp, k, ldm)))
    return fail(MF_ERR_ARG, "Y overlaps P or M");
  hipError_t err = launch_block_update(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy,
                                       static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "block update kernel launch");
  return MF_OK;
}

int64_t mf_block_update_norms_work(int64_t n, int k) {
  if (n < 0 || k < 1) return -1;
  const int64_t w = update_workgroups(n);
  return (w < 1 ? 1 : w) * (int64_t)k;
}

int mf_block_update_norms(int64_t n, int k, int kp, double alpha, const double* P, int64_t ldp,
                          const double* M, int ldm, double beta, double* Y, int64_t ldy,
                          double* norms2, double* work, int64_t work_len, void* stream) {
  if (!M || !norms2 || !work || (n > 0 && (!P || !Y)))
    return fail(MF_ERR_ARG, "P, M, Y, norms2 and work must be non-NULL");
  if (n < 0 || k < 1 || kp < 1 || ldp < kp || ldm < k || ldy < k)
    return fail(MF_ERR_ARG, "need n >= 0, k, kp >= 1, ldp >= kp, ldm >= k, ldy >= k");
  if (k > 128 || kp > 128 || !update_in_lds(k, kp))
    return fail(MF_ERR_UNSUPPORTED, "mf_block_update_norms takes k <= 128 and kp <= 128");
  if (work_len < mf_block_update_norms_work(n, k))
    return fail(MF_ERR_ARG, "work_len < mf_block_update_norms_work");
  const size_t ys = span_bytes(n, k, ldy), ns = (size_t)k * sizeof(double);
  const size_t ws = (size_t)work_len * sizeof(double);
  if (overlaps(Y, ys, P, span_bytes(n, kp, ldp)) || overlaps(Y, ys, M, span_bytes(kp, k, ldm)) ||
      overlaps(norms2, ns, Y, ys) || overlaps(norms2, ns, P, span_bytes(n, kp, ldp)) ||
      overlaps(norms2, ns, M, span_bytes(kp, k, ldm)) || overlaps(work, ws, Y, ys) ||
      overlaps(work, ws, P, span_bytes(n, kp, ldp)) || overlaps(work, ws, M, span_bytes(kp, k, ldm)) ||
      overlaps(work, ws, norms2, ns))
    return fail(MF_ERR_ARG, "Y, norms2 or work overlaps an operand or each other");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int64_t nw = update_workgroups(n);
  hipError_t err = hipSuccess;
  if (n > 0)
    err = launch_block_update(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, hs, work);
  if (err == hipSuccess) err = launch_chunk_sum(1, k, (int)nw, work, 1.0, 0.0, norms2, k, hs);
  if (err != hipSuccess) return hip_fail(err, "block update kernel launch");
  return MF_OK;
}

int mf_col_dots(int64_t n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                double* out, void* stream) {
  if (!out || (n > 0 && (!A || !B))) return fail(MF_ERR_ARG, "A, B and out must be non-NULL");
  if (n < 0 || k < 1 || lda < k || ldb < k) return fail(MF_ERR_ARG, "need n >= 0, k >= 1, ld >= k");
  hipError_t err = launch_col_dots(n, k, A, lda, B, ldb, out, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "column-dot kernel launch");
  return MF_OK;
}

int mf_axpby(int64_t n, int k, double a, const double* X, int64_t ldx, double b, double* Y,
             int64_t ldy, void* stream) {
  if (n > 0 && (!X || !Y)) return fail(MF_ERR_ARG, "X and Y must be non-NULL");
  if (n < 0 || k < 1 || ldx < k || ldy < k) return fail(MF_ERR_ARG, "need n >= 0, k >= 1, ld >= k");
  if (n == 0) return MF_OK;
  if (X != Y && overlaps(Y, span_bytes(n, k, ldy), X, span_bytes(n, k, ldx)))
    return fail(MF_ERR_ARG, "Y overlaps X without being equal to it");
  if (X == Y && ldx != ldy) return fail(MF_ERR_ARG, "in place needs ldx == ldy");
  hipError_t err = launch_axpby(n, k, a, X, ldx, b, Y, ldy, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "axpby kernel launch");
  return MF_OK;
}

int mf_jacobi(int64_t n, int k, const double* diag, const double* R, int64_t ldr, double* Z,
              int64_t ldz, void* stream) {
  if (n > 0 && (!diag || !R || !Z)) return fail(MF_ERR_ARG, "diag, R and Z must be non-NULL");
  if (n < 0 || k < 1 || ldr < k || ldz < k) return fail(MF_ERR_ARG, "need n >= 0, k >= 1, ld >= k");
  if (n == 0) return MF_OK;
  if (Z != R && overlaps(Z, span_bytes(n, k, ldz), R, span_bytes(n, k, ldr)))
    return fail(MF_ERR_ARG, "Z overlaps R without being equal to it");
  if (Z == R && ldz != ldr) return fail(MF_ERR_ARG, "in place needs ldz == ldr");
  hipError_t err = launch_jacobi(n, k, diag, R, ldr, Z, ldz, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "Jacobi kernel launch");
  return MF_OK;
}

int mf_spd_solve(int k, int m, const double* G, const double* S, double* X, int* status,
                 void* stream) {
  if (!G || !S || !X || !status) return fail(MF_ERR_ARG, "G, S, X and status must be non-NULL");
  if (k < 1 || m < 1) return fail(MF_ERR_ARG, "need k, m >= 1");
  if (k > spd_max_k() || m > 256) return fail(MF_ERR_UNSUPPORTED, "need k <= 128 and m <= 256");
  const size_t xs = span_bytes(k, m, m);
  if (overlaps(X, xs, G, span_bytes(k, k, k)) || overlaps(X, xs, S, xs))
    return fail(MF_ERR_ARG, "X overlaps G or S");
  hipError_t err = launch_spd_solve(k, m, G, S, X, status, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "SPD solve kernel launch");
  return MF_OK;
}

}  // extern "C"
