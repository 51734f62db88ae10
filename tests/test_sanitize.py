"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

1. The host linear algebra (csrc/hostla.cpp) built with g++ and both
   sanitizers into a stand-alone driver that exercises every routine over
   random and edge-case sizes (orders 1 and 2, band widths 0 .. 32, block
   Lanczos matrices of 1 .. 6 blocks) and checks the results itself.
2. The C-ABI driver (csrc/refl_api.cpp with hostla.cpp) compiled with the
   sanitizers on its host code only (-Xarch_host before each -fsanitize=;
   the device objects are the ordinary build's) and linked into a separate
   library, then called through ctypes on every path that runs without a
   device: defaults, status strings, argument checks, and handle creation,
   which reports the missing device.

Either run fails on any sanitizer report or a nonzero exit.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_24840_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
#include "hostla.h"
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
using namespace refl;

static unsigned long long st = 88172645463325252ull;
static double urand() {  // xorshift64, uniform in (-1, 1)
  st ^= st << 13; st ^= st >> 7; st ^= st << 17;
  return (double)(st >> 11) * 0x1.0p-52 - 1.0;
}
#define CHECK(c, ...) do { if (!(c)) { std::fprintf(stderr, __VA_ARGS__); std::fprintf(stderr, "\n"); return 1; } } while (0)

static int dense_eig(int n) {
  std::vector<double> A(n * n), w(n), Q(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) A[i * n + j] = A[j * n + i] = urand();
  CHECK(sym_eig_small(n, A.data(), w.data(), Q.data()) == 0, "eig failed n=%d", n);
  double scale = 0.0, worst = 0.0;
  for (double a : A) scale = std::fmax(scale, std::fabs(a));
  for (int c = 0; c < n; ++c) {
    if (c > 0) CHECK(w[c - 1] <= w[c], "not ascending n=%d", n);
    for (int i = 0; i < n; ++i) {
      double r = -w[c] * Q[i * n + c];
      for (int j = 0; j < n; ++j) r += A[i * n + j] * Q[j * n + c];
      worst = std::fmax(worst, std::fabs(r));
    }
  }
  CHECK(worst <= 1e-12 * n * (scale + 1.0), "eig residual %g n=%d", worst, n);
  return 0;
}

static int band(int n, int bw) {
  std::vector<double> Lb(n * (bw + 1), 0.0), dg(n), sb(n > 1 ? n - 1 : 1), work(n * (bw + 1));
  for (int i = 0; i < n; ++i)
    for (int t = 0; t <= bw && t <= i; ++t) Lb[i * (bw + 1) + t] = urand();
  band_tridiag(n, bw, Lb.data(), dg.data(), sb.data());
  double lo = tridiag_eigval(n, dg.data(), sb.data(), 0), hi = tridiag_eigval(n, dg.data(), sb.data(), n - 1);
  CHECK(lo <= hi, "eigval order n=%d bw=%d", n, bw);
  const int m = n / 2;
  const double x = tridiag_eigval(n, dg.data(), sb.data(), m);
  CHECK(tridiag_count_below(n, dg.data(), sb.data(), x - 1e-9) <= m, "count n=%d", n);
  const int c = band_count_below(n, bw, Lb.data(), x + 1e-7, work.data());
  CHECK(c == -1 || c >= m + 1, "band count %d < %d (n=%d bw=%d)", c, m + 1, n, bw);
  std::vector<double> y(n);
  const double r = band_inverse_iteration(n, bw, Lb.data(), x, 3, y.data());
  CHECK(std::isfinite(r), "inverse iteration n=%d", n);
  if (n >= 2) {                     // deflated against the first vector
    std::vector<double> y2(n);
    band_inverse_iteration(n, bw, Lb.data(), x, 2, y2.data(), y.data(), 1);
    double dot = 0.0;
    for (int i = 0; i < n; ++i) dot += y[i] * y2[i];
    CHECK(std::fabs(dot) <= 1e-8, "deflation n=%d dot=%g", n, dot);
  }
  return 0;
}

static int lanczos(int j, int b, int k) {
  std::vector<double> TA(j * b * b), TB(j * b * b, 0.0);
  for (int i = 0; i < j; ++i)
    for (int r = 0; r < b; ++r)
      for (int c = 0; c <= r; ++c) {
        TA[i * b * b + r + b * c] = TA[i * b * b + c + b * r] = urand();
        TB[i * b * b + c + b * r] = (c == r) ? 1.0 + std::fabs(urand()) : urand();  // upper
      }
  RitzCheck a, p2;
  ritz_check(j, b, k, TA.data(), TB.data(), true, a, nullptr);
  ritz_check(j, b, k, TA.data(), TB.data(), true, p2, &a);
  CHECK(a.th_k <= a.th_k1 && a.th_min <= a.th_k && a.th_k1 <= a.th_max, "ritz order j=%d b=%d", j, b);
  CHECK(std::fabs(a.th_k - p2.th_k) <= 1e-9 * (1 + std::fabs(a.th_k)), "warm bracket j=%d b=%d", j, b);
  const int nv = b < j * b ? b : j * b;
  std::vector<double> Y(j * b * nv);
  CHECK(ritz_vectors(j, b, TA.data(), TB.data(), nv, Y.data()) == 0, "ritz vectors j=%d b=%d", j, b);
  return 0;
}

int main() {
  for (int n : {1, 2, 3, 5, 8, 17, 32}) if (dense_eig(n)) return 1;
  for (int n : {1, 2, 5, 12, 40, 97})
    for (int bw : {0, 1, 3, 9, 16, 32})
      if (bw < n || bw == 0) { if (band(n, bw)) return 1; }
  for (int j : {1, 2, 6})
    for (int b : {1, 3, 9, 32}) {
      const int k = j * b > 1 ? std::min(j * b - 1, 5) : 0;
      if (k >= 1 && lanczos(j, b, k)) return 1;
    }
  std::printf("hostla sanitized driver: ok\n");
  return 0;
}
"""

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _clean(proc):
    text = proc.stdout + proc.stderr
    return proc.returncode == 0 and "AddressSanitizer" not in text and "runtime error" not in text


def test_hostla_under_asan_ubsan(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-I", CSRC, str(src),
                    os.path.join(CSRC, "hostla.cpp"), "-o", str(exe)], check=True)
    proc = subprocess.run([str(exe)], capture_output=True, text=True,
                          env=dict(os.environ, **SAN_ENV), timeout=300)
    assert _clean(proc), proc.stdout + proc.stderr
    assert "ok" in proc.stdout


CALLS = textwrap.dedent(r"""
    import ctypes, sys
    sys.path.insert(0, sys.argv[2])
    from paper_2605_24840_amd import refl
    lib = refl.load(sys.argv[1])
    p = refl.refl_params_default()
    for code in range(-1, 12):
        assert lib.refl_status_string(code)
    assert lib.refl_params_default(None) == 1
    assert lib.refl_create(None, 0, None) == 1
    h = ctypes.c_void_p()
    assert lib.refl_create(ctypes.byref(h), 0, None) == 2      # no device here
    assert lib.refl_create(ctypes.byref(h), -1, None) == 2
    assert lib.refl_destroy(None) == 1
    assert lib.refl_sign(None, 4, None, 4, ctypes.byref(p), None, 4, None) == 1
    assert lib.refl_sign_apply(None, 4, None, 4, ctypes.byref(p), 1, None, 4, None, 4, None) == 1
    assert lib.refl_apply(None, 4, None, 4, 1, None, 4, None, 4) == 1
    assert lib.refl_sign_batched(None, 1, None, None, None, None, None, None, None, None) == 1
    assert lib.refl_sign_batched_workspace_size(None, 1, None, None, None) == 1
    assert lib.refl_workspace_size(None, 4, ctypes.byref(p), None) == 1
    assert lib.refl_estimate_shift(None, 4, None, 4, 1, 0, 0, None, None, None, None, None) == 1
    assert lib.refl_sign_grad(None, 4, None, 4, ctypes.byref(p), None, 4, None, 4, None, None, 4, None) == 1
    assert lib.refl_policy_create(None, None, None) == 1
    assert lib.refl_policy_destroy(None) == 1
    assert lib.refl_last_error(None) == b"NULL handle"
    print("driver sanitized calls: ok")
""")


def test_driver_host_code_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2605_24840_amd import build as libbuild
    rt = subprocess.run([HIPCC, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        import glob
        found = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not found:
            pytest.skip("clang ASan runtime not found")
        rt = found[0]
    objs = []
    for name in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, name)
        if name.endswith(".hip"):
            obj = os.path.join(libbuild.BUILD, name + ".o")
            if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(path):
                os.makedirs(libbuild.BUILD, exist_ok=True)
                obj = libbuild._compile(path)
            objs.append(obj)
        elif name.endswith(".cpp"):
            obj = str(tmp_path / (name + ".o"))
            flags = [f for f in libbuild.FLAGS if f != "-O3"]
            subprocess.run([HIPCC] + flags + ["-O1", "-g", "-fno-omit-frame-pointer",
                                              "-Xarch_host", "-fsanitize=address",
                                              "-Xarch_host", "-fsanitize=undefined",
                                              "-c", path, "-o", obj], check=True, capture_output=True)
            objs.append(obj)
    so = str(tmp_path / "librefl_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-shared-libsan", "-o", so] + objs, check=True, capture_output=True)
    script = tmp_path / "calls.py"
    script.write_text(CALLS)
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=rt, HIP_VISIBLE_DEVICES="")
    proc = subprocess.run([sys.executable, str(script), so, ROOT], capture_output=True, text=True,
                          env=env, timeout=300)
    assert _clean(proc), proc.stdout + proc.stderr
    assert "ok" in proc.stdout
