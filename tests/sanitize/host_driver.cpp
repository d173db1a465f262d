// Sanitizer driver for the host side of libthzspec (argument checks, plan
// shapes, bin frequencies, the batch's job table and the fault-injection
// paths), built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host by tests/test_sanitizers.py.  It needs no GPU: every call returns
// before device work (invalid arguments) or is a pure host helper, and the
// allocation paths are cut by TZ_FAULT=alloc before hipMalloc.  Exit status
// 0 when every status and value is the expected one.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "thzspec.h"

static int bad = 0;
#define EXPECT(c)                                                     \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "%s:%d: failed: %s (%s)\n", __FILE__, __LINE__, #c, tz_last_error()); \
      bad = 1;                                                        \
    }                                                                 \
  } while (0)

int main() {
  tz_opts o;
  tz_opts_init(&o);
  void *fx = (void *)0x1000, *fX = (void *)0x2000;  // stand-ins: never dereferenced on these paths
  tz_c64 W = {cos(0.01), -sin(0.01)}, A = {1.0, 0.0}, Z = {0.0, 0.0};

  // helpers of eqs. (3)-(5), (22)-(25)
  tz_c64 w, a;
  EXPECT(czt_band(20e12, 0.2e12, 2.5e12, 4096, &w, &a) == TZ_OK);
  EXPECT(czt_band(20e12, 2.5e12, 0.2e12, 4096, &w, &a) == TZ_EINVAL);
  EXPECT(fft_zero_count(10e12, 500, 0.5e9) > 0 && fft_zero_count(10e12, 500, 0.0) == -1);
  EXPECT(czt_points_for_resolution(8000, 100, 1000, 128) == 14);
  EXPECT(zoom_short_length(20e12, 0.2e12, 2.5e12, 4096, 6) > 0 && zoom_short_length(0, 1, 2, 3, 4) == -1);
  int64_t L = 0, blocks = 0;
  for (int64_t N : {1LL, 300LL, 4096LL, 16000LL, 1000000LL, (1LL << 24)})
    for (int64_t M : {1LL, 1000LL, 9000LL, 300000LL}) {
      const tz_status st = czt_plan_shape(N, M, &L, &blocks);
      EXPECT(st == TZ_OK || st == TZ_EUNSUPPORTED);
      if (st == TZ_OK) EXPECT(L >= 1 && blocks >= 1);
    }
  EXPECT(czt_plan_shape(0, 5, &L, &blocks) == TZ_EINVAL);

  // bin frequencies of every plan kind
  tz_plan_params p;
  memset(&p, 0, sizeof p);
  p.N = 1000;
  p.M = 777;
  p.n_zeros = 1048;
  p.W = W;
  p.A = A;
  p.fs = 20e12;
  p.f1 = 0.2e12;
  p.f2 = 2.5e12;
  p.fs_hz = 20000000000000LL;
  p.f1_hz = 200000000000LL;
  p.f2_hz = 2500000000000LL;
  p.D = 6;
  std::vector<double> f(2048);
  for (int kind : {TZ_PLAN_FFT_ZEROPAD, TZ_PLAN_CZT, TZ_PLAN_CZT_BAND_EXACT, TZ_PLAN_ZOOM}) {
    p.kind = kind;
    EXPECT(tz_bin_freqs(&p, nullptr, f.data()) == TZ_OK);
  }
  o.flags = TZ_HALF;
  p.kind = TZ_PLAN_FFT_ZEROPAD;
  EXPECT(tz_bin_freqs(&p, &o, f.data()) == TZ_OK && f[1024] == 10e12);
  o.flags = 0;
  p.kind = TZ_PLAN_IFFT;
  EXPECT(tz_bin_freqs(&p, nullptr, f.data()) == TZ_EINVAL);

  // invalid arguments are refused before device work
  EXPECT(fft_zeropad(nullptr, 10, 0, fX, &o) == TZ_EINVAL);
  EXPECT(fft_zeropad(fx, 0, 0, fX, &o) == TZ_EINVAL);
  EXPECT(fft_zeropad(fx, 10, -1, fX, &o) == TZ_EINVAL);
  EXPECT(czt(fx, 10, 0, W, A, fX, &o) == TZ_EINVAL);
  EXPECT(czt(fx, 10, 5, Z, A, fX, &o) == TZ_EINVAL);
  EXPECT(czt_band_exact(fx, 10, 5, 0, 0, 1, fX, &o) == TZ_EINVAL);
  EXPECT(zoom_fft(fx, 100, 20e12, 2e12, 1e12, 64, 4, fX, &o) == TZ_EINVAL);
  EXPECT(ifft(fx, 0, fX, &o) == TZ_EINVAL);
  tz_czt_axis ax[2] = {{8, 4, W, A}, {0, 4, W, A}};
  EXPECT(czt_nd(fx, 2, ax, fX, &o) == TZ_EINVAL);
  EXPECT(czt_nd(fx, 4, ax, fX, &o) == TZ_EINVAL);
  tz_plan *pl = nullptr;
  p.kind = 9;
  EXPECT(tz_plan_create(&p, nullptr, &pl) == TZ_EINVAL && pl == nullptr);
  EXPECT(tz_plan_execute(nullptr, fx, fX, nullptr, nullptr) == TZ_EINVAL);
  EXPECT(tz_plan_execute_static(nullptr, fx, fX, nullptr) == TZ_EINVAL);

  // the batch's job table: invalid jobs, then valid ones up to the first
  // allocation, which the injected fault refuses
  std::vector<tz_job> jobs(3);
  for (int i = 0; i < 3; ++i) {
    memset(&jobs[i], 0, sizeof(tz_job));
    jobs[i].kind = i == 1 ? TZ_JOB_ZOOM : TZ_JOB_CZT;
    jobs[i].N = 500 + 4000 * i;
    jobs[i].M = 300 + 2000 * i;
    jobs[i].D = 6;
    jobs[i].fs_hz = 20000000000000LL;
    jobs[i].f1_hz = 200000000000LL;
    jobs[i].f2_hz = 2500000000000LL;
    jobs[i].in_offset = 10000 * i;
    jobs[i].out_offset = 10000 * i;
  }
  tz_batch *b = nullptr;
  jobs[2].M = 0;
  EXPECT(tz_batch_create(jobs.data(), 3, nullptr, &b) == TZ_EINVAL && b == nullptr);
  jobs[2].M = 20000;
  setenv("TZ_FAULT", "alloc", 1);
  EXPECT(tz_batch_create(jobs.data(), 3, nullptr, &b) == TZ_ENOMEM && b == nullptr);
  EXPECT(fft_zeropad(fx, 100, 28, fX, &o) == TZ_ENOMEM);
  unsetenv("TZ_FAULT");
  EXPECT(tz_batch_wait(nullptr, 1.0) == TZ_EINVAL);
  EXPECT(strlen(tz_version()) > 0);
  char buf[16];
  EXPECT(tz_batch_describe(nullptr, buf, sizeof buf) == -1);
  tz_release_plans();
  if (!bad) printf("host driver: ok\n");
  return bad;
}
