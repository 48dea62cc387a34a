// Travel time and source gradient of one row in FP64 from the network
// output (o, do/du_src): T = T0 f with T0 = |x - s|/v0 and f = softplus(o)/ln 2
// (o = 0 is the homogeneous medium of Sec. 2.1); dT/dx = f (x - s)/(v0 |x - s|)
// + T0 sigmoid(o)/ln 2 do/dx, with do/dx = do/du_src / h.  Two FP64
// divisions per row (1/|x - s| and 1/(1 + e^-|o|)); 1/v0 and 1/ln 2 are
// constants.
#pragma once
#include "net_rows.h"

namespace spider {

constexpr double kInvLn2 = 1.4426950408889634073599246810019;  // 1 / ln 2

__device__ inline void assemble_tt(const NetView& net, const double x[3], const double s[3],
                                   const RowOut& no, double& T, double g[3]) {
  const double d0 = x[0] - s[0], d1 = x[1] - s[1], d2 = x[2] - s[2];
  const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double inv_dist = 1.0 / dist;
  const double T0 = dist * net.inv_v0;
  const double o = (double)no.o;
  const double ex = exp(-fabs(o));             // one exponential for both
  const double sp = fmax(o, 0.0) + log1p(ex);  // softplus
  const double r1 = 1.0 / (1.0 + ex);
  const double sg = o >= 0.0 ? r1 : ex * r1;   // sigmoid
  const double f = sp * kInvLn2;
  T = T0 * f;
  const double a = f * net.inv_v0 * inv_dist;
  const double bsc = T0 * sg * kInvLn2;
  g[0] = a * d0 + bsc * ((double)no.d0 * net.inv_half[0]);
  g[1] = a * d1 + bsc * ((double)no.d1 * net.inv_half[1]);
  g[2] = a * d2 + bsc * ((double)no.d2 * net.inv_half[2]);
}

}  // namespace spider
