/* Dart throwing for the variable-density Poisson-disc masks of synth/inputs.py.
 *
 * One pass over the candidates in their given (seeded) order: candidate t at grid point
 * (ii[t], jj[t]) is accepted when no point already occupied lies strictly closer than
 * dmin[t] grid cells; the occupied set starts as the fully sampled centre (occ0).  The
 * window, the distance test and the acceptance order are those of the Python loop in
 * poisson_disc_plane, which this replaces for speed only (the masks are identical).
 *
 * Built by the package's build step with the host C compiler; input generation only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t pd_throw(int32_t n0, int32_t n1, const uint8_t* occ0, int64_t ncand, const int32_t* ii,
                 const int32_t* jj, const double* dmin, int64_t* acc) {
  uint8_t* occ = (uint8_t*)malloc((size_t)n0 * (size_t)n1);
  if (!occ) return -1;
  memcpy(occ, occ0, (size_t)n0 * (size_t)n1);
  int64_t na = 0;
  for (int64_t t = 0; t < ncand; ++t) {
    const int32_t i = ii[t], j = jj[t];
    const double d = dmin[t];
    const int32_t w = (int32_t)ceil(d);
    const int32_t i0 = i - w > 0 ? i - w : 0, i1 = i + w + 1 < n0 ? i + w + 1 : n0;
    const int32_t j0 = j - w > 0 ? j - w : 0, j1 = j + w + 1 < n1 ? j + w + 1 : n1;
    int hit = 0;
    for (int32_t a = i0; a < i1 && !hit; ++a)
      for (int32_t b = j0; b < j1; ++b)
        if (occ[(size_t)a * n1 + b]) {
          const int64_t di = a - i, dj = b - j;
          if ((double)(di * di + dj * dj) < d * d) { hit = 1; break; }
        }
    if (hit) continue;
    occ[(size_t)i * n1 + j] = 1;
    acc[na++] = t;
  }
  free(occ);
  return na;
}
