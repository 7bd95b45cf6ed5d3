// Batched launches: one launch of a V-cycle operator covers that operator's
// work for every problem of a batch of independent problems (uneven sizes
// included).  Each problem contributes a job (its grid, vectors and
// workgroup range); the kernels look their job up by workgroup index, so a
// launch is as wide as all problems together and a V-cycle of the batch is
// one chain of launches instead of one chain per problem.
#include "common.h"

namespace mvpf {

int batch_job_blocks(int op, const BJob& j, int threads) {
  switch (op) {
    case BOP_CONVERT:
    case BOP_FINISH: return vec_job_blocks(j.g);
    case BOP_PBJ_ZERO:
    case BOP_DEFECT_SPLIT:
    case BOP_PBJ_LOWER:
    case BOP_DEFECT_LOWER:
    case BOP_ROW_SMALL_PBJ:
    case BOP_ROW_SMALL_DEFECT: return bsr_job_blocks(op, j.g);
    case BOP_RESTRICT: return (j.g2.Npad + 255) / 256;
    case BOP_PROLONG: return (j.g.Npad + 255) / 256;
    case BOP_COARSE: return (int)(((int64_t)NDOF * j.g.N + 3) / 4);
    case BOP_MF_ELEMENT:
    case BOP_MF_GATHER_PBJ:
    case BOP_MF_GATHER_DEFECT:
    case BOP_MF_OUTER_ELEMENT:
    case BOP_MF_OUTER_GATHER: return mf_job_blocks(op, j.g, threads);
    default: return 0;
  }
}

template <typename T, typename TZ>
void launch_batch(int op, const BJob* jobs_dev, int njobs, int total_blocks, hipStream_t s, int threads) {
  if (njobs <= 0 || total_blocks <= 0) return;
  switch (op) {
    case BOP_CONVERT:
    case BOP_FINISH: launch_vec_batch<T, TZ>(op, jobs_dev, njobs, total_blocks, s); break;
    case BOP_RESTRICT:
    case BOP_PROLONG: launch_transfer_batch<T>(op, jobs_dev, njobs, total_blocks, s); break;
    case BOP_COARSE: launch_coarse_solve_batch<T>(jobs_dev, njobs, total_blocks, s); break;
    case BOP_MF_ELEMENT:
    case BOP_MF_GATHER_PBJ:
    case BOP_MF_GATHER_DEFECT: launch_mf_batch<T>(op, jobs_dev, njobs, total_blocks, s, threads); break;
    case BOP_MF_OUTER_ELEMENT:
    case BOP_MF_OUTER_GATHER: launch_mf_outer_batch<TZ>(op, jobs_dev, njobs, total_blocks, s, threads); break;
    default: launch_bsr_batch<T>(op, jobs_dev, njobs, total_blocks, s); break;
  }
}
template void launch_batch<float, float>(int, const BJob*, int, int, hipStream_t, int);
template void launch_batch<float, double>(int, const BJob*, int, int, hipStream_t, int);
template void launch_batch<double, double>(int, const BJob*, int, int, hipStream_t, int);

}  // namespace mvpf
