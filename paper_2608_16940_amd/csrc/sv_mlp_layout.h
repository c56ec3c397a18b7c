// Layout of the cost-model MLP's flat parameter vector (sv_mlp.h):
// W1[nin][hid], b1[hid], W2[hid][hid], b2[hid], W3[hid], b3[1].
#pragma once

namespace sv {

struct MlpOffsets {
  int w1, b1, w2, b2, w3, b3, total;
};

inline MlpOffsets mlp_offsets(int nin, int hid) {
  MlpOffsets o;
  o.w1 = 0;
  o.b1 = o.w1 + nin * hid;
  o.w2 = o.b1 + hid;
  o.b2 = o.w2 + hid * hid;
  o.w3 = o.b2 + hid;
  o.b3 = o.w3 + hid;
  o.total = o.b3 + 1;
  return o;
}

}  // namespace sv
