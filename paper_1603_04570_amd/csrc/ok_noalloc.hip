// ok_residual_noalloc: the Newton residual for callers that cannot allocate.
//
// Its scratch (the constants-table record, the residual-assembly fields t1,
// t2, the quadrature field G, the reduction partials and the norm) lives in
// one file-scope device array, `scratch`, of kScratchBytes.  Host code never
// passes the array's name to a kernel or a copy: the name is a host-side
// stand-in.  On the first call on a device, with that device current, the
// array's device address is taken with hipGetSymbolAddress and kept per
// device; every later use goes through that address.  Every call on a device
// shares its array, so calls are serialised per device by a host mutex (and
// each call synchronises its stream before returning, so no two calls'
// kernels overlap on one device).  Nothing in the scratch must start at zero:
// every kernel fully writes what the next one reads.
#include <cstring>
#include <mutex>

#include "engine.h"

using namespace okd;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

struct DeviceScratch {
  std::mutex mu;
  char* ptr = nullptr;  // device address of `scratch` on this device
};
DeviceScratch g_scratch[kMaxDevices];

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch for a grid of `nodes` nodes: constants record, t1, t2, G,
// reduction partials, norm.
size_t scratch_need(int64_t nodes) {
  return up256(sizeof(InstCoef)) + 3 * up256((size_t)nodes * sizeof(double)) +
         up256(kMaxRedBlocks * sizeof(double)) + up256(8 * sizeof(double));
}

}  // namespace

extern "C" int ok_residual_noalloc(const ok_params* p, const double* u, const double* w,
                                   const double* un, const double* wn, double* F,
                                   double* h_norm, void* stream) {
  std::string why;
  if (validate_params(p, why)) return OK_E_INVALID;
  if (!u || !w || !un || !F || (p->theta < 1.0 && !wn)) return OK_E_INVALID;
  for (const void* q : {(const void*)u, (const void*)w, (const void*)un, (const void*)F})
    if ((uintptr_t)q & 7) return OK_E_INVALID;
  if (wn && ((uintptr_t)wn & 7)) return OK_E_INVALID;
  const Grid g = make_grid(p->dim, p->n);
  if (scratch_need(g.nodes) > kScratchBytes) return OK_E_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return OK_E_HIP;
  DeviceScratch& ds = g_scratch[dev];
  std::lock_guard<std::mutex> lock(ds.mu);
  if (!ds.ptr) {
    void* a = nullptr;
    if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return OK_E_HIP;
    ds.ptr = (char*)a;
  }
  // carve the scratch: constants, t1, t2, G, partials, norm
  char* q = ds.ptr;
  InstCoef* coef = (InstCoef*)q;
  q += up256(sizeof(InstCoef));
  const size_t fb = up256((size_t)g.nodes * sizeof(double));
  double* t1 = (double*)q;
  double* t2 = (double*)(q + fb);
  double* G = (double*)(q + 2 * fb);
  q += 3 * fb;
  double* part = (double*)q;
  q += up256(kMaxRedBlocks * sizeof(double));
  double* nrm = (double*)q;

  InstCoef hc;
  Grid lev[kMaxLevels];
  int L = 0;
  instance_constants(*p, hc, lev, L);
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(coef, &hc, sizeof(hc), hipMemcpyHostToDevice, st) != hipSuccess)
    return OK_E_HIP;
  const Batch B{1, coef, nullptr};
  const Vec<const double> wnv{(p->theta < 1.0 || wn) ? wn : nullptr, 0};
  hipError_t e = residual_launch(g, B, Vec<const double>{u, 0}, Vec<const double>{w, 0},
                                 Vec<const double>{un, 0}, wnv, Vec<double>{F, 0},
                                 Vec<double>{t1, 0}, Vec<double>{t2, 0}, Vec<double>{G, 0},
                                 Vec<double>{part, 0}, Vec<double>{nrm, 0}, st);
  double hn[2] = {0.0, 0.0};
  if (e == hipSuccess) e = hipMemcpyAsync(hn, nrm, sizeof(hn), hipMemcpyDeviceToHost, st);
  // the host record hc and hn must outlive their copies: complete the stream
  const hipError_t es = hipStreamSynchronize(st);
  if (e != hipSuccess || es != hipSuccess) return OK_E_HIP;
  if (h_norm) *h_norm = hn[1];
  return OK_SUCCESS;
}
