// Host-side checks of the C ABI layer under AddressSanitizer and
// UndefinedBehaviorSanitizer, with no GPU: argument validation of fca_init
// and fca_batch_init, option parsing on a context built on the host, error
// strings, and the tune-cache file parser on malformed files.  Built with
// g++ from the host sources only (tests/test_host_sanitizer.py); paths that
// would reach a kernel or the device are not called.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "fca_internal.h"

static int g_fail = 0;
#define EXPECT(cond, what)                                   \
  do {                                                       \
    if (!(cond)) {                                           \
      std::printf("FAIL %s (line %d)\n", what, __LINE__);    \
      ++g_fail;                                              \
    }                                                        \
  } while (0)

static void init_validation() {
  alignas(16) static float buf[64];
  const fca_c64* x = reinterpret_cast<const fca_c64*>(buf);
  const float* v = buf;
  const fca_c64* x_odd = reinterpret_cast<const fca_c64*>(reinterpret_cast<const char*>(buf) + 4);
  const float* v_odd = reinterpret_cast<const float*>(reinterpret_cast<const char*>(buf) + 2);
  fca_ctx* c = reinterpret_cast<fca_ctx*>(1);
  struct Case { fca_method m; int F, N, I, J; const fca_c64* x; const float* v; const fca_c64* R; fca_status want; };
  const Case cases[] = {
      {(fca_method)7, 4, 64, 3, 3, x, v, nullptr, FCA_ERR_ARG},        // unknown method
      {FCA_METHOD_AS, 0, 64, 3, 3, x, v, nullptr, FCA_ERR_ARG},        // F = 0
      {FCA_METHOD_AS, 4, -1, 3, 3, x, v, nullptr, FCA_ERR_ARG},        // N < 0
      {FCA_METHOD_AS, 4, 64, 0, 3, x, v, nullptr, FCA_ERR_ARG},        // I = 0
      {FCA_METHOD_AS, 4, 64, 9, 3, x, v, nullptr, FCA_ERR_UNSUPPORTED},// I > 8
      {FCA_METHOD_AS, 4, 64, 3, 10, x, v, nullptr, FCA_ERR_UNSUPPORTED},
      {FCA_METHOD_AS, 4, 2, 3, 3, x, v, nullptr, FCA_ERR_ARG},         // N < I
      {FCA_METHOD_AS, 1 << 20, 1 << 12, 8, 9, x, v, nullptr, FCA_ERR_ARG},  // too large
      {FCA_METHOD_AS, 2147483647, 2147483647, 8, 9, x, v, nullptr, FCA_ERR_ARG},
      {FCA_METHOD_AS, 4, 64, 3, 3, nullptr, v, nullptr, FCA_ERR_ARG},  // NULL x
      {FCA_METHOD_AS, 4, 64, 3, 3, x, nullptr, nullptr, FCA_ERR_ARG},  // NULL v0
      {FCA_METHOD_AS, 4, 64, 3, 3, x_odd, v, nullptr, FCA_ERR_ARG},    // misaligned complex
      {FCA_METHOD_AS, 4, 64, 3, 3, x, v_odd, nullptr, FCA_ERR_ARG},    // misaligned float
      {FCA_METHOD_AS, 4, 64, 3, 3, x, v, x, FCA_ERR_ARG},              // R0 with AS
      {FCA_METHOD_EM, 4, 64, 3, 3, x, v, x_odd, FCA_ERR_ARG},          // misaligned R0
  };
  for (const Case& k : cases) {
    c = reinterpret_cast<fca_ctx*>(1);
    const fca_status st = fca_init(&c, k.m, k.F, k.N, k.I, k.J, k.x, k.v, k.v, x, k.R, nullptr);
    EXPECT(st == k.want, "fca_init status");
    EXPECT(c == nullptr, "fca_init leaves *out NULL on failure");
    const char* e = fca_last_error(nullptr);
    EXPECT(e && std::strlen(e) > 0, "fca_init error string");
  }
  EXPECT(fca_init(nullptr, FCA_METHOD_AS, 4, 64, 3, 3, x, v, v, x, nullptr, nullptr) == FCA_ERR_ARG, "NULL out");
}

static fca_ctx* host_ctx(fca_method m) {
  fca_ctx* c = new fca_ctx();
  c->method = m; c->F = 4; c->N = 64; c->I = 3; c->J = 3;
  c->s.K = 1; c->s.p_step = 0.1f; c->split = 2; c->autotune = 1; c->last_waves = -1; c->last_bpw = -1;
  return c;
}

static void options() {
  fca_ctx* c = host_ctx(FCA_METHOD_AS);
  struct Opt { const char* key; long long value; fca_status want; };
  const Opt set[] = {
      {"K", 1, FCA_OK}, {"K", 64, FCA_OK}, {"K", 0, FCA_ERR_ARG}, {"K", 65, FCA_ERR_ARG},
      {"K", -9223372036854775807LL, FCA_ERR_ARG}, {"K", 9223372036854775807LL, FCA_ERR_ARG},
      {"p_update", 4, FCA_OK}, {"p_update", 5, FCA_ERR_ARG}, {"p_update", -1, FCA_ERR_ARG}, {"p_update", 0, FCA_OK},
      {"check_finite", 1, FCA_OK}, {"check_finite", 2, FCA_ERR_ARG},
      {"path", 2, FCA_OK}, {"path", 3, FCA_ERR_ARG},
      {"waves", 4, FCA_OK}, {"waves", 3, FCA_ERR_ARG}, {"waves", 8, FCA_ERR_ARG},
      {"bins_per_wg", 2, FCA_OK}, {"bins_per_wg", 3, FCA_ERR_ARG},
      {"autotune", 0, FCA_OK}, {"autotune", 2, FCA_ERR_ARG},
      {"split_streams", 4, FCA_OK}, {"split_streams", 0, FCA_ERR_ARG}, {"split_streams", 5, FCA_ERR_ARG},
      {"sums_mfma", 2, FCA_OK}, {"sums_mfma", 1, FCA_OK}, {"sums_mfma", 3, FCA_ERR_ARG}, {"sums_mfma", -2, FCA_ERR_ARG},
      {"", 1, FCA_ERR_ARG}, {"no such option", 1, FCA_ERR_ARG}, {"Kx", 1, FCA_ERR_ARG},
  };
  for (const Opt& o : set) {
    EXPECT(fca_set_option(c, o.key, o.value) == o.want, o.key);
    EXPECT(std::strlen(fca_last_error(c)) < 4096, "error string length");
  }
  long long v = -7;
  const char* keys[] = {"K", "p_update", "check_finite", "path", "waves", "bins_per_wg", "autotune",
                        "split_streams", "sums_mfma", "last_waves", "last_bins_per_wg"};
  for (const char* k : keys) EXPECT(fca_get_option(c, k, &v) == FCA_OK, k);
  EXPECT(fca_get_option(c, "K", &v) == FCA_OK && v == 64, "K read back");
  EXPECT(fca_get_option(c, "sums_mfma", &v) == FCA_OK && v == 1, "sums_mfma read back");
  EXPECT(fca_get_option(c, "nope", &v) == FCA_ERR_ARG, "unknown get");
  EXPECT(fca_get_option(c, nullptr, &v) == FCA_ERR_ARG, "NULL key get");
  EXPECT(fca_get_option(c, "K", nullptr) == FCA_ERR_ARG, "NULL value get");
  EXPECT(fca_set_option(c, nullptr, 1) == FCA_ERR_ARG, "NULL key set");
  EXPECT(fca_set_option(nullptr, "K", 1) == FCA_ERR_ARG, "NULL ctx set");
  double d = 0;
  EXPECT(fca_set_option_f64(c, "p_step", 0.5) == FCA_OK, "p_step");
  EXPECT(fca_set_option_f64(c, "p_step", 0.0) == FCA_ERR_ARG, "p_step 0");
  EXPECT(fca_set_option_f64(c, "p_step", 1e300) == FCA_ERR_ARG, "p_step huge");
  EXPECT(fca_set_option_f64(c, "p_step", 0.0 / 0.0) == FCA_ERR_ARG, "p_step NaN");
  EXPECT(fca_get_option_f64(c, "p_step", &d) == FCA_OK && d == 0.5, "p_step read back");
  EXPECT(fca_set_option_f64(c, "K", 1.0) == FCA_ERR_ARG, "integer key as real");
  delete c;
  fca_ctx* e = host_ctx(FCA_METHOD_EM);
  EXPECT(fca_set_option(e, "p_update", 1) == FCA_ERR_STATE, "p_update on an EM context");
  EXPECT(fca_set_option(e, "p_update", 0) == FCA_OK, "p_update 0 on an EM context");
  delete e;
  EXPECT(std::strlen(fca_last_error(nullptr)) > 0, "global error string");
}

static void batch_validation() {
  fca_batch* b = reinterpret_cast<fca_batch*>(1);
  alignas(16) static float buf[64];
  const int F[2] = {4, 4}, N[2] = {64, 64}, I[2] = {3, 9}, J[2] = {3, 3};
  const fca_c64* xs[2] = {reinterpret_cast<const fca_c64*>(buf), reinterpret_cast<const fca_c64*>(buf)};
  const float* vs[2] = {buf, buf};
  EXPECT(fca_batch_init(nullptr, 2, F, N, I, J, xs, vs, vs, xs, nullptr) == FCA_ERR_ARG, "batch NULL out");
  EXPECT(fca_batch_init(&b, 0, F, N, I, J, xs, vs, vs, xs, nullptr) == FCA_ERR_ARG && b == nullptr, "batch n_mix 0");
  EXPECT(fca_batch_init(&b, 2, nullptr, N, I, J, xs, vs, vs, xs, nullptr) == FCA_ERR_ARG, "batch NULL F");
  EXPECT(fca_batch_init(&b, 2, F, N, I, J, xs, vs, vs, xs, nullptr) == FCA_ERR_UNSUPPORTED, "batch I = 9");
  EXPECT(std::strlen(fca_batch_last_error(nullptr)) > 0, "batch error string");
  EXPECT(fca_batch_set_option(nullptr, "graph", 1) == FCA_ERR_ARG, "batch NULL set");
}

static void tune_cache() {
  char path[] = "/tmp/fca_tune_cache_XXXXXX";
  const int fd = mkstemp(path);
  EXPECT(fd >= 0, "mkstemp");
  if (fd < 0) return;
  FILE* f = fdopen(fd, "w");
  std::fprintf(f, "good\t1 2\nno tab at all\nbad numbers\tx y\none number\t3\n\t4 4\n");
  std::string longkey(3000, 'k');
  std::fprintf(f, "%s\t5 6\n", longkey.c_str());  // longer than the reader's line buffer
  std::fputc('\0', f);
  std::fprintf(f, "after nul\t7 8\ngood\t9 10\n");  // a later line wins
  std::fprintf(f, "no newline at end\t11 12");
  std::fclose(f);
  setenv("FASTFCA_TUNE_CACHE", path, 1);
  int a = -1, bb = -1;
  EXPECT(fca::tune_cache_get("good", &a, &bb) && a == 9 && bb == 10, "later line wins");
  EXPECT(!fca::tune_cache_get("no tab at all", &a, &bb), "line without tab");
  EXPECT(!fca::tune_cache_get("bad numbers", &a, &bb), "non-numeric values");
  EXPECT(!fca::tune_cache_get("one number", &a, &bb), "one value");
  EXPECT(fca::tune_cache_get("no newline at end", &a, &bb) && a == 11 && bb == 12, "last line without newline");
  (void)fca::tune_cache_get(longkey, &a, &bb);  // split by the line buffer: any result, no memory error
  fca::tune_cache_put("with\ttab", 1, 1);
  fca::tune_cache_put("with\nnewline", 1, 1);
  EXPECT(!fca::tune_cache_get("with\ttab", &a, &bb), "key with a tab is not stored");
  fca::tune_cache_put("fresh key", 13, 14);
  EXPECT(fca::tune_cache_get("fresh key", &a, &bb) && a == 13 && bb == 14, "put then get");
  FILE* g = std::fopen(path, "a");  // another process appends
  std::fprintf(g, "other process\t15 16\n");
  std::fclose(g);
  EXPECT(fca::tune_cache_get("other process", &a, &bb) && a == 15, "re-read after growth");
  setenv("FASTFCA_TUNE_CACHE", "/nonexistent/dir/cache", 1);
  EXPECT(!fca::tune_cache_get("good", &a, &bb), "unreadable file");
  fca::tune_cache_put("x", 1, 2);  // unwritable: no effect
  setenv("FASTFCA_TUNE_CACHE", "", 1);
  EXPECT(!fca::tune_cache_get("good", &a, &bb), "empty variable");
  unsetenv("FASTFCA_TUNE_CACHE");
  std::remove(path);
}

int main() {
  init_validation();
  options();
  batch_validation();
  tune_cache();
  if (g_fail) {
    std::printf("%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("HOST SANITIZER OK\n");
  return 0;
}
