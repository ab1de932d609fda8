// C ABI of the Chebyshev-filter building blocks (include/mfcheb.h).
#include "mf_internal.h"
#include "mfcheb.h"
#include "mfrefine.h"

using namespace mf;

namespace {

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* a0 = static_cast<const char*>(a);
  const char* b0 = static_cast<const char*>(b);
  return a0 < b0 + bn && b0 < a0 + an;
}

}  // namespace

extern "C" {

int mf_gll_mass(mf_operator* handle, int inv_sqrt, double* out, void* stream) {
  if (!handle || !out) return fail(MF_ERR_ARG, "operator and out must be non-NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (op->refined) {
    // the lumped mass of every cell, then C^T (row sums of C^T M C), then m^{-1/2}
    hipError_t err = launch_gll_mass_map(*op, out, s);
    if (err == hipSuccess && op->nsets > 0) err = launch_constraints_condense(*op, out, 1, 1, s);
    if (err == hipSuccess && inv_sqrt) err = launch_inv_sqrt(out, op->ndofs, s);
    if (err != hipSuccess) return hip_fail(err, "lumped mass kernel launch");
    return MF_OK;
  }
  if (!op->box) return fail(MF_ERR_UNSUPPORTED, "the lumped mass is built for axis-aligned cells");
  hipError_t err = launch_gll_mass(*op, inv_sqrt, out, s);
  if (err != hipSuccess) return hip_fail(err, "lumped mass kernel launch");
  return MF_OK;
}

int mf_cheb_step(mf_operator* handle, const double* D, const double* Y, const double* Xp,
                 double* Out, int nvec, int64_t ld, double a, double b, double c, void* stream) {
  if (!handle || !D || !Y || !Out) return fail(MF_ERR_ARG, "operator, D, Y and Out must be non-NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (nvec < 1 || ld < nvec) return fail(MF_ERR_ARG, "need nvec >= 1 and ld >= nvec");
  if (!op->box) return fail(MF_ERR_UNSUPPORTED, "the Chebyshev step is built for axis-aligned cells");
  const size_t span = (size_t)((op->ndofs - 1) * ld + nvec) * sizeof(double);
  const size_t dspan = (size_t)op->ndofs * sizeof(double);
  if (overlaps(Out, span, Y, span) || overlaps(Out, span, D, dspan))
    return fail(MF_ERR_ARG, "Out overlaps Y or D");
  if (Xp && Xp != Out && overlaps(Out, span, Xp, span))
    return fail(MF_ERR_ARG, "Xp must be Out itself or not overlap it");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t err = launch_cheb_init(*op, Y, Xp, Out, ld, nvec, b, c, s);
  if (err != hipSuccess) return hip_fail(err, "Chebyshev init kernel launch");
  const ChebArgs ca{D, Xp, a, b, c};
  err = launch_apply_cheb(*op, Y, Out, ld, nvec, ca, s);
  if (err != hipSuccess) return hip_fail(err, "Chebyshev step kernel launch");
  return MF_OK;
}

int mf_cheb_step_constrained(mf_operator* handle, const double* D, const double* Y,
                             const double* Xp, double* Out, int nvec, int64_t ld, double a,
                             double b, double c, double* work, void* stream) {
  if (!handle || !D || !Y || !Out || !work)
    return fail(MF_ERR_ARG, "operator, D, Y, Out and work must be non-NULL");
  if (nvec < 1 || ld < nvec) return fail(MF_ERR_ARG, "need nvec >= 1 and ld >= nvec");
  Operator* op = reinterpret_cast<Operator*>(handle);
  const size_t span = (size_t)((op->ndofs - 1) * ld + nvec) * sizeof(double);
  const size_t dspan = (size_t)op->ndofs * sizeof(double);
  const size_t wspan = 2 * (size_t)op->ndofs * nvec * sizeof(double);
  if (overlaps(Out, span, Y, span) || overlaps(Out, span, D, dspan) ||
      overlaps(Out, span, work, wspan))
    return fail(MF_ERR_ARG, "Out overlaps Y, D or work");
  if (overlaps(work, wspan, Y, span) || overlaps(work, wspan, D, dspan) ||
      (Xp && overlaps(work, wspan, Xp, span)))
    return fail(MF_ERR_ARG, "work overlaps an input");
  if (Xp && Xp != Out && overlaps(Out, span, Xp, span))
    return fail(MF_ERR_ARG, "Xp must be Out itself or not overlap it");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* W = work;
  double* V = work + op->ndofs * (int64_t)nvec;
  hipError_t err = launch_scale_rows(op->ndofs, nvec, D, Y, ld, W, s);  // W = D Y
  if (err != hipSuccess) return hip_fail(err, "row scaling kernel launch");
  if (int st = mf_apply_constrained(handle, W, V, nvec, nvec, nvec, stream)) return st;
  err = launch_cheb_combine(op->ndofs, nvec, D, V, Y, Xp, Out, ld, a, b, c, s);
  if (err != hipSuccess) return hip_fail(err, "Chebyshev combine kernel launch");
  return MF_OK;
}

int64_t mf_sym_eig_work(int k) {
  if (k < 1 || k > eig_blocked_max_k()) return -1;
  return k <= eig_max_k() ? 0 : sym_eig_blocked_work(k);
}

int mf_sym_eig(int k, const double* A, int64_t lda, double* w, double* V, int64_t ldv,
               double vpow, int* status, double* work, int64_t work_len, void* stream) {
  if (!A || !w || !V || !status) return fail(MF_ERR_ARG, "A, w, V and status must be non-NULL");
  if (k < 1 || k > eig_blocked_max_k()) return fail(MF_ERR_UNSUPPORTED, "need 1 <= k <= 2048");
  if (lda < k || ldv < k) return fail(MF_ERR_ARG, "need lda, ldv >= k");
  const size_t as = (size_t)((k - 1) * lda + k) * sizeof(double);
  const size_t vs = (size_t)((k - 1) * ldv + k) * sizeof(double);
  const size_t ws = (size_t)k * sizeof(double);
  if (overlaps(V, vs, A, as) || overlaps(w, ws, A, as) || overlaps(w, ws, V, vs))
    return fail(MF_ERR_ARG, "w and V must not overlap A or each other");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (k <= eig_max_k()) {
    hipError_t err = launch_sym_eig(k, A, lda, w, V, ldv, vpow, status, s);
    if (err != hipSuccess) return hip_fail(err, "eigen-decomposition kernel launch");
    return MF_OK;
  }
  const int64_t need = sym_eig_blocked_work(k);
  if (!work || work_len < need)
    return fail(MF_ERR_ARG, "k > 64 needs a work array of mf_sym_eig_work(k) doubles");
  const size_t wks = (size_t)need * sizeof(double);
  if (overlaps(work, wks, A, as) || overlaps(work, wks, V, vs) || overlaps(work, wks, w, ws) ||
      overlaps(work, wks, status, sizeof(int)))
    return fail(MF_ERR_ARG, "work must not overlap A, w, V or status");
  hipError_t err = launch_sym_eig_blocked(k, A, lda, w, V, ldv, vpow, status, work, s);
  if (err != hipSuccess) return hip_fail(err, "block Jacobi kernel launch");
  return MF_OK;
}

}  // extern "C"
