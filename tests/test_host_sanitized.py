"""The library's host code under AddressSanitizer and UBSan, on a machine
without a GPU (tests/hostcheck): the host translation units are built for the
host only and linked against a stand-in for the HIP runtime that checks every
stream, event, graph and allocation call against the programming model's
rules, and every kernel launch's parameters against the buffers the kernel
would touch.  The driver calls every entry point, including chunk batches
that are created, replayed on two streams, autotuned six times in a row,
tuned before their first launch and destroyed with launches still queued."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests", "hostcheck"))


@pytest.fixture(scope="module")
def hostcheck(tmp_path_factory):
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc is not installed")
    import build as hcbuild
    return hcbuild.build(str(tmp_path_factory.mktemp("hostcheck")))


def _run(exe, **env):
    e = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1", **env)
    return subprocess.run([exe], capture_output=True, text=True, timeout=600, env=e)


def test_host_code_is_clean_under_sanitizers(hostcheck):
    r = _run(hostcheck)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "hostcheck: OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_stub_catches_a_graph_destroyed_while_launched(hostcheck, tmp_path):
    """The stand-in itself is checked: a program that destroys an executable
    graph right after launching it, without waiting, must be stopped."""
    src = tmp_path / "bad.cpp"
    src.write_text(r'''
#include "hostcheck.h"
int main() {
  hipStream_t s, o;
  hipEvent_t f, j;
  (void)hipStreamCreateWithFlags(&s, 0);
  (void)hipStreamCreateWithFlags(&o, 0);
  (void)hipEventCreateWithFlags(&f, 0);
  (void)hipEventCreateWithFlags(&j, 0);
  (void)hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  (void)hipEventRecord(f, s);
  (void)hipStreamWaitEvent(o, f, 0);
  hc::kernel_launch(o, "k");
  (void)hipEventRecord(j, o);
  (void)hipStreamWaitEvent(s, j, 0);
  hipGraph_t g;
  (void)hipStreamEndCapture(s, &g);
  hipGraphExec_t x;
  (void)hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphLaunch(x, nullptr);
  (void)hipGraphExecDestroy(x);
  return 0;
}
''')
    import build as hcbuild
    out = os.path.dirname(hostcheck)
    obj = str(tmp_path / "bad.o")
    hcbuild._compile(str(src), obj)
    exe = str(tmp_path / "bad")
    subprocess.run([hcbuild.tool("clang++"), "-fsanitize=address,undefined", obj, os.path.join(out, "hip_stub.o"),
                    os.path.join(out, "fatbin_blobs.o"), "-o", exe], check=True, capture_output=True)
    r = _run(exe)
    assert r.returncode != 0
    assert "hipGraphExecDestroy while a launch of it" in r.stderr
