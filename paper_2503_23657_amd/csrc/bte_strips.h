// Strip position of a wave slot in the 1D/2D rows-per-lane schedule, tracked
// incrementally chunk by chunk (host and device).
//
// Slot r of R owns strips r, r+R, ...; strip s starts at clock s*du, so a lane
// at lane-relative clock q works on strip s, column v = q - s*du, when
// 0 <= v < nx. Consecutive strips of one slot start R*du apart; when no slot
// owns more than one strip (n_strip <= R) the slot simply holds strip r.
#pragma once

#if defined(__HIPCC__)
#define BTE_HD __host__ __device__ __attribute__((always_inline))
#else
#define BTE_HD
#endif

namespace bte {

struct StripTrack {
  int s, v;       // strip and column at the current clock
  int period;     // R*du when slots own several strips, 0 otherwise

  BTE_HD void init(int q, int r, int R, int du, int n_strip) {
    if (n_strip <= R) {
      period = 0;
      s = r;
      v = q - r * du;
      return;
    }
    period = R * du;
    const int a = q - r * du;
    const int m = a >= 0 ? a / period : -((-a + period - 1) / period);
    s = r + m * R;
    v = q - s * du;
  }
  // clock += dq (0 < dq <= du)
  BTE_HD void advance(int dq, int R) {
    v += dq;
    if (period && v >= period) {
      v -= period;
      s += R;
    }
  }
  BTE_HD bool valid(int n_strip, int nx) const { return s >= 0 && s < n_strip && v >= 0 && v < nx; }
};

}  // namespace bte
