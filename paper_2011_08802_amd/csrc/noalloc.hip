// mvpf_residual_noalloc: the residual of mvpf_residual with no device memory
// allocated by the call or by the library on its behalf.  Its scratch -- the
// per-Gauss-point gradients of one slab of element layers and the partial
// sums of the free-dof norm -- lives in a file-scope device array of fixed
// size; each GPU holds its own copy of the array (at its own address) until
// the process ends.
#include <cmath>
#include <mutex>
#include <string>

#include "common.h"

using namespace mvpf;

namespace {

// Scratch layout (doubles): [0, RED) partial sums of the norm, [RED, QP0)
// the reduced value, [QP0, end) Gauss-point gradients of one slab,
// QP_GRAD * 8 values per element.
constexpr int64_t SCRATCH_DOUBLES = (int64_t)8 << 20;  // 64 MiB
constexpr int64_t RED = MAX_RED_BLOCKS;
constexpr int64_t QP0 = RED + 4096;
constexpr int64_t NE_CAP = ((SCRATCH_DOUBLES - QP0) / (QP_GRAD * 8)) / TILE * TILE;

static_assert(QP0 % 32 == 0, "the Gauss-point slab starts 256-byte aligned");

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
double* g_ptr[MAX_DEVICES] = {};

// The device address of this GPU's copy of `scratch` (looked up once per
// device, with that device current).  In host code the array's name is only
// a host-side stand-in; kernels and copies get this address.
int scratch_ptr(mvpf_problem* p, double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    p->err = std::string("residual_noalloc: no usable current device: ") + hipGetErrorString(e);
    return MVPF_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      p->err = std::string("residual_noalloc: hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return MVPF_EDEVICE;
    }
    g_ptr[dev] = (double*)ptr;
  }
  *out = g_ptr[dev];
  return 0;
}

int check(mvpf_problem* p, const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    p->err = std::string(where) + ": " + hipGetErrorString(e);
    return MVPF_EDEVICE;
  }
  return 0;
}

}  // namespace

extern "C" {

int mvpf_residual_noalloc_max_layer(void) { return (int)((NE_CAP - TILE) / 2); }

int mvpf_residual_noalloc(mvpf_problem* p, double* R, double* norm_free) {
  if (!p) return MVPF_EINVAL;
  Level& L0 = p->lev[0];
  const Grid& g = L0.g;
  // a slab holds at least two element layers (one of them the halo layer)
  if (2 * (int64_t)g.nx * g.ny + TILE > NE_CAP) {
    p->err = "residual_noalloc: nx * ny = " + std::to_string((int64_t)g.nx * g.ny) +
             " elements per layer exceeds the fixed scratch (at most " +
             std::to_string(mvpf_residual_noalloc_max_layer()) + ")";
    return MVPF_EINVAL;
  }
  double* base = nullptr;
  int rc = scratch_ptr(p, &base);
  if (rc) return rc;
  double* part = base;
  double* red = base + RED;
  double* qp = base + QP0;
  hipStream_t s = p->stream;
  const double depth = p->have_system ? p->sys_depth : p->depth;
  // the same kernels and slab logic as mvpf_residual; every scratch value
  // read is written earlier in the same call, so nothing needs clearing
  launch_dirichlet_masks(g, p->load, depth, L0.mask, L0.target, s);
  for (const Chunk& ck : make_chunks(g, NE_CAP)) {
    launch_qp(g, ck, L0.state, p->card, p->pade, p->mixing, qp, false, s);
    launch_residual_gather(g, ck, L0.state, qp, p->card, p->R, s);
  }
  if (p->load.kind == MVPF_LOAD_SPHERE)
    launch_contact_residual(g, make_sphere(g, p->load, depth), L0.state, p->R, s);
  if ((rc = check(p, "residual_noalloc"))) return rc;
  if (norm_free) {
    const int nb = red_blocks((int64_t)g.N * NDOF);
    launch_free_norm_partial(g, p->R, L0.mask, part, s);
    launch_reduce(1, nb, part, red, 0, s);
    if ((rc = check(p, "residual_noalloc norm"))) return rc;
    hipError_t e = hipMemcpyAsync(p->hhost, red, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      p->err = std::string("residual_noalloc: norm read-back failed: ") + hipGetErrorString(e);
      return MVPF_EDEVICE;
    }
    *norm_free = std::sqrt(p->hhost[0]);
  }
  if (R) launch_soa_to_interleaved(g, p->R, NDOF, 0, NDOF, R, s);
  if ((rc = check(p, "residual_noalloc"))) return rc;
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    p->err = std::string("residual_noalloc: ") + hipGetErrorString(e);
    return MVPF_EDEVICE;
  }
  return 0;
}

}  // extern "C"
