// The dispatcher's 16 input features, computed the same way on the host (the drivers' decisions) and on
// the device (the batched launch's per-graph decisions).  Not part of the public C-ABI.
#pragma once
#include "bmlp_internal.h"

namespace bmlp {

//  0 log2(1+n)/16            1 log2(1+m)/24             2 log2(1+m/n)/8 (mean degree)
//  3 log2(1+maxdeg/(1+m/n))/8 (degree skew)             4 nonempty rows / n
//  5 log2(1+k)/16            6 min(k/n, 4)              7 context: 1 composition, 0.5 closure computed
//                                                         anyway (batched launch), 0 selection
//  8 call-level query (1) or round-level query (0)       9 round / 64
// 10 |delta| / (k n)         11 |visited| / (k n)        12 log2(1+|delta|)/32
// 13 min(|delta| / |previous delta|, 16) / 16            14 log2(1 + |delta| m/n)/40 (edges to visit)
// 15 reflexive answer (0/1)
__host__ __device__ inline void make_features(float* f, double n_, double m, double maxdeg, double nonempty, double k,
                                              float context, int call_level, int round, double delta,
                                              double prev_delta, double vis, int reflexive) {
  const double n = n_ > 1.0 ? n_ : 1.0, kk = k > 1.0 ? k : 1.0;
  const double deg = m / n;
  f[0] = (float)(log2(1.0 + n) / 16.0);
  f[1] = (float)(log2(1.0 + m) / 24.0);
  f[2] = (float)(log2(1.0 + deg) / 8.0);
  f[3] = (float)(log2(1.0 + maxdeg / (1.0 + deg)) / 8.0);
  f[4] = (float)(nonempty / n);
  f[5] = (float)(log2(1.0 + k) / 16.0);
  f[6] = (float)(k / n < 4.0 ? k / n : 4.0);
  f[7] = context;
  f[8] = call_level ? 1.f : 0.f;
  f[9] = (float)(round / 64.0);
  f[10] = (float)(delta / (kk * n));
  f[11] = (float)(vis / (kk * n));
  f[12] = (float)(log2(1.0 + delta) / 32.0);
  const double ratio = delta / (prev_delta > 1.0 ? prev_delta : 1.0);
  f[13] = (float)((ratio < 16.0 ? ratio : 16.0) / 16.0);
  f[14] = (float)(log2(1.0 + delta * deg) / 40.0);
  f[15] = reflexive ? 1.f : 0.f;
}

}  // namespace bmlp
