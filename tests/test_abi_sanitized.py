"""The ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer: the library's
sources and a host-only driver (tests/sanitize/abi_driver.cpp) are built with both
sanitizers on the host side only, and the driver walks every argument-error path, the
workspace sizes and the status strings.  No device work is launched, so no GPU is needed."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2011_11082_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer",
       "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


def test_abi_host_paths_under_sanitizers(tmp_path):
    try:
        cc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    common = [c for c in B.COMMON if c != "-O3"]
    jobs = []
    for src, extra in B.SOURCES.items():
        jobs.append([cc, *common, *extra, *SAN, "-c", os.path.join(B.CSRC, src),
                     "-o", str(tmp_path / (os.path.splitext(src)[0] + ".o"))])
    jobs.append([cc, *common, "-x", "hip", *SAN, "-c",
                 os.path.join(HERE, "sanitize", "abi_driver.cpp"),
                 "-o", str(tmp_path / "abi_driver.o")])
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), jobs))
    for r, c in zip(results, jobs):
        assert r.returncode == 0, f"{' '.join(c)}\n{r.stderr[-2000:]}"
    exe = str(tmp_path / "abi_driver")
    objs = [str(p) for p in sorted(tmp_path.glob("*.o"))]
    r = subprocess.run([cc, f"--offload-arch={B.ARCH}", *objs, "-o", exe,
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-3000:]
