// Host-only pieces shared by every translation unit of libsv: the calling
// thread's last error message, and the test for gates that only permute
// their qubits.  Plain C++, no HIP.
#include <string>

#include "sv_guard.h"

namespace sv {

namespace {
thread_local std::string g_err;
}  // namespace

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

// True when G maps each basis state |c> to |pi(c)>, pi moving bit j of c to
// bit perm[j] (a permutation of the block's qubits), with exact 0/1 entries.
bool qubit_permutation(const double *G, int k, int *perm) {
  const int D = 1 << k;
  for (int i = 0; i < D * D; ++i)
    if (G[2 * i + 1] != 0.0 || (G[2 * i] != 0.0 && G[2 * i] != 1.0)) return false;
  int used = 0;
  for (int j = 0; j < k; ++j) {
    int row = -1;
    for (int r = 0; r < D; ++r)
      if (G[2 * (r * D + (1 << j))] == 1.0) {
        if (row >= 0) return false;
        row = r;
      }
    if (row <= 0 || (row & (row - 1)) || (used & row)) return false;
    used |= row;
    perm[j] = __builtin_ctz(unsigned(row));
  }
  for (int c = 0; c < D; ++c) {
    int r = 0;
    for (int j = 0; j < k; ++j) r |= ((c >> j) & 1) << perm[j];
    for (int rr = 0; rr < D; ++rr)
      if (G[2 * (rr * D + c)] != (rr == r ? 1.0 : 0.0)) return false;
  }
  return true;
}

}  // namespace sv

extern "C" const char *sv_last_error(void) { return sv::g_err.c_str(); }
