// Cost-model MLP on the host: parameter counts and the FP64 forward pass the
// planner scores blocks with.  Plain C++, no HIP.
#include <cstdint>
#include <vector>

#include "sv_guard.h"
#include "sv_mlp.h"
#include "sv_mlp_layout.h"

using namespace sv;

extern "C" {

int sv_mlp_param_count(int nin, int hid) { return mlp_offsets(nin, hid).total; }

int64_t sv_mlp_cache_floats(int hid, int batch) { return 4 * int64_t(hid) * batch; }

int sv_mlp_forward_host(const float *p, int nin, int hid, const float *x, int batch, double *y) {
  return guard([&]() -> int {
    if (!p || !x || !y || nin < 1 || hid < 1 || batch < 0) {
      set_error("bad host mlp argument");
      return SV_ERR_ARG;
    }
    const MlpOffsets o = mlp_offsets(nin, hid);
    std::vector<double> h1(static_cast<size_t>(hid)), h2(static_cast<size_t>(hid));
    for (int r = 0; r < batch; ++r) {
      const float *xr = x + int64_t(r) * nin;
      for (int u = 0; u < hid; ++u) {
        double a = p[o.b1 + u];
        for (int i = 0; i < nin; ++i) a += double(xr[i]) * double(p[o.w1 + i * hid + u]);
        h1[size_t(u)] = a > 0 ? a : 0;
      }
      for (int u = 0; u < hid; ++u) {
        double a = p[o.b2 + u];
        for (int i = 0; i < hid; ++i) a += h1[size_t(i)] * double(p[o.w2 + i * hid + u]);
        h2[size_t(u)] = a > 0 ? a : 0;
      }
      double a = p[o.b3];
      for (int u = 0; u < hid; ++u) a += h2[size_t(u)] * double(p[o.w3 + u]);
      y[r] = a;
    }
    return SV_OK;
  });
}

}  // extern "C"
