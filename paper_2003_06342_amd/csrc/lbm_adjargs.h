// Argument block of the 2-D adjoint kernels (shared with the C ABI).
#pragma once

#include "lbm_adjoint.h"

namespace lbm {

using adj::NodeAdjIn;
using adj::NodeConst;
using adj::NodeIn;
using adj::NodeOut;

enum { LL_PHI = 0, LL_GX, LL_GY, LL_LAP, LL_UX, LL_UY, LL_D, LL_N };

template <class Real>
struct AdjArgs {
  Real* lA;        // 27 planes: lambda of the stored populations
  Real* lphip;     // lambda of phi_prev
  Real* lqp;       // lambda of q_prev
  Real* lP;        // 27 planes: lambda of the pulled populations (scratch)
  Real* lloc;      // LL_N planes (scratch)
  Real* fphi;      // forward phi and u of the step being reversed
  Real* fux;
  Real* fuy;
  Real* lTw[2][2];  // wall-temperature gradient accumulators [axis][side]
  NodeConst<Real> nc;
};

}  // namespace lbm
