// Host-only exercise of the C ABI's validation, footprint and error paths, for
// a build of the runtime under AddressSanitizer and UndefinedBehaviorSanitizer
// (host code only; no GPU is touched: every call here fails or finishes before
// its first device call).  Prints one line per group and "host checks ok".
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "pasd.h"

static int fails = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      printf("FAILED %s:%d %s\n", __FILE__, __LINE__, #cond);        \
      ++fails;                                                       \
    }                                                                \
  } while (0)

static pasd_config cfg3(long a, long b, long c, long r) {
  pasd_config cfg;
  pasd_config_init(&cfg);
  cfg.order = 3;
  cfg.dims[0] = a;
  cfg.dims[1] = b;
  cfg.dims[2] = c;
  for (int n = 0; n < 3; ++n) cfg.ranks[n] = r;
  return cfg;
}

int main() {
  // defaults and validation codes
  pasd_config c = cfg3(50, 50, 50, 5);
  CHECK(pasd_validate(&c) == PASD_OK);
  CHECK(pasd_validate(NULL) == PASD_ERR_INVALID_ARG);
  CHECK(strlen(pasd_last_error()) > 0);
  for (int order = -1; order <= PASD_MAX_ORDER + 2; ++order) {
    pasd_config d = c;
    d.order = order;
    for (int n = 3; n < PASD_MAX_ORDER; ++n) {
      d.dims[n] = 2;
      d.ranks[n] = 1;
    }
    const int rc = pasd_validate(&d);
    CHECK((order >= 2 && order <= PASD_MAX_ORDER) ? rc == PASD_OK : rc == PASD_ERR_INVALID_ARG);
  }
  const long ranks[] = {-3, 0, 1, 16, 17, 64, 65, 1000};
  for (long r : ranks) {
    pasd_config d = cfg3(100, 100, 100, r);
    const int rc = pasd_validate(&d);
    CHECK(r >= 1 && r <= 64 ? rc == PASD_OK : rc != PASD_OK);
  }
  {
    pasd_config d = c;
    d.lambda[1] = NAN;
    CHECK(pasd_validate(&d) == PASD_ERR_INVALID_ARG);
    d = c;
    d.mu0 = -1;
    CHECK(pasd_validate(&d) == PASD_ERR_INVALID_ARG);
    d = c;
    d.tol = INFINITY;
    CHECK(pasd_validate(&d) == PASD_ERR_INVALID_ARG);
    d = c;
    d.flags = 1 << 20;
    CHECK(pasd_validate(&d) == PASD_ERR_INVALID_ARG);
    d = c;
    d.precision = 99;
    CHECK(pasd_validate(&d) == PASD_ERR_INVALID_ARG);
    d = cfg3(1L << 31, 2, 2, 1);
    CHECK(pasd_validate(&d) != PASD_OK);
    d = cfg3(1L << 14, 1L << 14, 1L << 14, 1);
    CHECK(pasd_validate(&d) == PASD_ERR_UNSUPPORTED);
  }
  printf("validation ok\n");
  // footprints grow with size and precision, and match across calls
  size_t b64 = 0, b32 = 0, b64b = 0;
  CHECK(pasd_footprint(&c, &b64) == PASD_OK);
  c.precision = PASD_FP32;
  CHECK(pasd_footprint(&c, &b32) == PASD_OK);
  c.precision = PASD_FP64;
  CHECK(pasd_footprint(&c, &b64b) == PASD_OK && b64b == b64 && b32 < b64);
  CHECK(pasd_footprint(&c, NULL) == PASD_ERR_INVALID_ARG);
  for (int order = 2; order <= PASD_MAX_ORDER; ++order) {
    pasd_config d;
    pasd_config_init(&d);
    d.order = order;
    for (int n = 0; n < order; ++n) {
      d.dims[n] = 3 + n;
      d.ranks[n] = 1 + n % 3;
    }
    size_t b = 0;
    CHECK(pasd_footprint(&d, &b) == PASD_OK && b > 0);
  }
  printf("footprint ok\n");
  // create, batch and destroy: argument errors before any device call
  pasd_ctx* ctx = (pasd_ctx*)0x1;
  double buf[8] = {0};
  pasd_config bad = cfg3(50, 50, 50, 0);
  CHECK(pasd_create(&bad, buf, 0, &ctx) == PASD_ERR_INVALID_ARG && ctx == NULL);
  CHECK(pasd_create(&c, NULL, 0, &ctx) == PASD_ERR_INVALID_ARG && ctx == NULL);
  CHECK(pasd_create(&c, buf, 0, NULL) == PASD_ERR_INVALID_ARG);
  pasd_info info;
  CHECK(pasd_step(NULL, 1) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_solve(NULL, &info) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_query(NULL, &info) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_get_result(NULL, buf, buf, 0) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_export(NULL, PASD_Q_E, 0, buf, 0) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_import(NULL, PASD_Q_E, 0, buf, 0) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_step_batch(NULL, 2, 1) == PASD_ERR_INVALID_ARG);
  pasd_ctx* none[2] = {NULL, NULL};
  CHECK(pasd_step_batch(none, 2, 1) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_step_batch(none, 0, 1) == PASD_OK);
  CHECK(pasd_query_batch(NULL, 1, &info) == PASD_ERR_INVALID_ARG);
  CHECK(pasd_profile(NULL, 1, NULL, NULL) == PASD_ERR_INVALID_ARG);
  pasd_destroy(NULL);
  printf("error paths ok\n");
  if (fails == 0) printf("host checks ok\n");
  return fails == 0 ? 0 : 1;
}
