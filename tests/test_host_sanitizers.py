"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with both sanitizers on its host code (device code unchanged) and the C ABI
tests run against it in a child process that preloads the ASan runtime: handle creation and
destruction, size queries, every host-side validation path.  A heap error, a use after free, an
out-of-bounds host access or undefined behaviour ends the child with a report.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHECK_LOADED = r"""
import sys
sys.path.insert(0, {root!r})
from paper_1910_13247_amd import _lib, build
assert _lib.LIB_PATH == build.SAN_LIB, _lib.LIB_PATH
_lib.lib()
maps = open("/proc/self/maps").read()
assert build.SAN_LIB in maps, "sanitized library not mapped"
assert "libclang_rt.asan" in maps, "ASan runtime not mapped"
print("sanitized library loaded")
"""


def _sanitized_library():
    from paper_1910_13247_amd import build
    newest = max(os.path.getmtime(s) for s in build.sources() + [os.path.join(ROOT, "include", "mfq.h")])
    if not os.path.exists(build.SAN_LIB) or os.path.getmtime(build.SAN_LIB) < newest:
        build.build(sanitize=True)
    return build


def test_abi_under_host_sanitizers():
    build = _sanitized_library()
    env = build.sanitizer_env()
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", _CHECK_LOADED.format(root=ROOT)], env=env, capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr
