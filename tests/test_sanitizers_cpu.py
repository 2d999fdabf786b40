"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The library's host side (argument validation, map set-up and teardown,
  every entry point's checks) is rebuilt with ASan + UBSan on its host code
  (device code unchanged) and driven by tests/abi_args_driver.c, which calls
  every entry point with invalid arguments and the creation path (on a machine
  without a GPU it fails at the first device call and must free what it
  took); leaks are reported too.
* The CPU oracle is rebuilt with ASan + UBSan and the oracle's pin tests run
  against it in a child interpreter with the sanitizer runtime preloaded.

Any out-of-bounds access, use of freed memory, leak (library) or undefined
behaviour on these paths fails the run.  The builds are cached under
_build/sanitize, keyed by the sources and flags."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
CSRC = os.path.join(ROOT, "paper_2311_00626_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _stamp(paths, flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _cached_build(name, sources, flags, cmd):
    """Runs cmd unless OUT/name exists from the same sources and flags."""
    os.makedirs(OUT, exist_ok=True)
    target = os.path.join(OUT, name)
    stamp_file = target + ".stamp"
    stamp = _stamp(sources, flags)
    if os.path.exists(target) and os.path.exists(stamp_file) and open(stamp_file).read() == stamp:
        return target
    subprocess.run(cmd, check=True, cwd=OUT, capture_output=True)
    with open(stamp_file, "w") as f:
        f.write(stamp)
    return target


@pytest.fixture(scope="module")
def asan_library():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_2311_00626_amd import build as hip_build
    srcs = [os.path.join(CSRC, s) for s in hip_build.SOURCES]
    deps = srcs + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + \
        [os.path.join(ROOT, "include", "tsdf.h")]
    flags = [f for f in hip_build.FLAGS if not f.startswith("-O")] + ["-O1"] + HOST_SAN
    cmd = [HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", "libtsdf_asan.so"]
    return _cached_build("libtsdf_asan.so", deps, flags, cmd)


def test_abi_argument_paths_under_asan_ubsan(asan_library):
    driver_src = os.path.join(ROOT, "tests", "abi_args_driver.c")
    flags = ["-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer"]
    cmd = [CLANG, *flags, "-I", os.path.join(ROOT, "include"), driver_src, "-L", OUT, "-ltsdf_asan",
           f"-Wl,-rpath,{OUT}", "-lm", "-o", "abi_args_driver"]
    exe = _cached_build("abi_args_driver", [driver_src, asan_library], flags, cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout


def test_oracle_pins_under_asan_ubsan():
    src = os.path.join(ROOT, "oracle", "tsdf_oracle.c")
    deps = [src] + [os.path.join(ROOT, "oracle", f) for f in ("oracle_impl.h", "sensor_model_impl.h",
                                                              "tsdf_oracle.h")]
    from oracle import build as oracle_build
    flags = [f for f in oracle_build.CFLAGS if f != "-O2"] + ["-O1", "-g", "-fsanitize=address,undefined",
                                                              "-fno-sanitize-recover=undefined",
                                                              "-fno-omit-frame-pointer"]
    lib = _cached_build("libtsdf_oracle_asan.so", deps, flags,
                        ["gcc", *flags, "-o", "libtsdf_oracle_asan.so", src, "-lm"])
    runtime = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
               for n in ("libasan.so", "libubsan.so")]
    assert all(os.path.isabs(p) and os.path.exists(p) for p in runtime), runtime
    env = dict(os.environ, LD_PRELOAD=":".join(runtime), ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSDF_ORACLE_LIB=lib)
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_oracle_pins.py", "test_oracle_lidar.py",
                                                       "test_oracle_dda.py", "test_oracle_threads.py",
                                                       "test_oracle_sensor_model.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout
