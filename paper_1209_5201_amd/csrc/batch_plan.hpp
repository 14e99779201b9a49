// Grouping of batched cases by storage format (host code, no HIP).
#pragma once

namespace lbm {

// Stable grouping of n cases by format code fmt[i] in [0, nfmt): the cases
// of format p take the positions start[p] .. start[p + 1] - 1, in input
// order; pos[i] is the position of case i.  start has nfmt + 1 entries,
// start[nfmt] = n.  Returns false (and writes nothing) if a code is out of
// range.
inline bool plan_groups(const int* fmt, int n, int nfmt, int* start, int* pos) {
  for (int i = 0; i < n; ++i)
    if (fmt[i] < 0 || fmt[i] >= nfmt) return false;
  int m = 0;
  for (int p = 0; p < nfmt; ++p) {
    start[p] = m;
    for (int i = 0; i < n; ++i)
      if (fmt[i] == p) pos[i] = m++;
  }
  start[nfmt] = m;
  return true;
}

}  // namespace lbm
