// Dispatch of the fused apply by polynomial degree, and the zero-fill kernel.
#include "mf_internal.h"
#include "sf_common.h"

namespace mf {

namespace {

// Y rows [0, nrows) x columns [0, ncols) := 0.  A kernel rather than a memset
// so that it also clears strided (ld > ncols) outputs and can be captured in a
// graph.
__global__ void zero_rows_kernel(double* __restrict__ Y, int64_t nrows, int ncols, int64_t ld) {
  const int64_t total = nrows * ncols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ncols, c = i % ncols;
    Y[r * ld + c] = 0.0;
  }
}

}  // namespace

hipError_t launch_zero_rows(double* Y, int64_t nrows, int ncols, int64_t ld, hipStream_t s) {
  const int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Y, nrows, ncols, ld);
  return hipGetLastError();
}

bool apply_f64_supported(int p, int q) {
  if (p < 1 || p > kMaxP || q < p + 1 || q > p + kMaxQExtra) return false;
  return f64_lds_bytes(p + 1, q, 1) <= 64 * 1024;
}

int choose_vtile_f64(int np, int nq, int nvec) {
  // enough (vector, pencil) work items to occupy 256 threads in the
  // pencil stages, as many as the 64 KiB LDS budget allows
  int vt = 256 / (nq * nq);
  if (vt < 1) vt = 1;
  while (vt > 1 && f64_lds_bytes(np, nq, vt) > 64 * 1024) --vt;
  if (vt > nvec) vt = nvec;
  return vt;
}

hipError_t launch_apply_f64(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_f64_p<1>(op, a, s);
    case 2: return launch_apply_f64_p<2>(op, a, s);
    case 3: return launch_apply_f64_p<3>(op, a, s);
    case 4: return launch_apply_f64_p<4>(op, a, s);
    case 5: return launch_apply_f64_p<5>(op, a, s);
    case 6: return launch_apply_f64_p<6>(op, a, s);
    case 7: return launch_apply_f64_p<7>(op, a, s);
    case 8: return launch_apply_f64_p<8>(op, a, s);
    case 9: return launch_apply_f64_p<9>(op, a, s);
    case 10: return launch_apply_f64_p<10>(op, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
