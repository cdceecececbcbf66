"""AddressSanitizer and UndefinedBehaviorSanitizer on host code.

The oracle, the multithreaded CPU peel and the input generators (gcc), and
the host code of libabcore (hipcc; device code is compiled as usual, only the
host side is instrumented) are rebuilt with both sanitizers into a temporary
folder and exercised by the CPU tests in a child process, with the
sanitizer runtime preloaded (the interpreter itself is not instrumented, so
leak checking is off).  Any report aborts the child.  Canaries with a heap
overflow and a signed overflow check that the runtime does report."""
import concurrent.futures
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GCC_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fPIC", "-shared"]


def _gcc_runtime():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()


def _clang_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def _run(cmd, env_extra, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def _build_helpers(out):
    libs = {}
    for env, src, comp, extra in (
            ("ABC_ORACLE_LIB", "oracle/abcore_oracle.c", "gcc", ["-std=c99"]),
            ("ABC_CPU_PEEL_LIB", "cpu_peel/cpu_peel.c", "gcc", ["-std=c99", "-fopenmp"]),
            ("ABC_BIGRAPH_GEN_LIB", "bigraph_gen/gen.cpp", "g++", ["-std=c++17", "-fopenmp"])):
        path = os.path.join(out, os.path.basename(src).split(".")[0] + ".so")
        subprocess.run([comp, *GCC_SAN, *extra, os.path.join(ROOT, src), "-o", path],
                       check=True)
        libs[env] = path
    return libs


def test_sanitizer_canaries(tmp_path):
    src = tmp_path / "canary.c"
    src.write_text(
        "#include <stdlib.h>\n"
        "int heap(int i) { int *p = malloc(4 * sizeof(int)); int v = p[i]; free(p); return v; }\n"
        "int add(int a, int b) { return a + b; }\n")
    pre = {"LD_PRELOAD": _gcc_runtime()}
    # each sanitizer alone (UBSan's object-size check would otherwise report
    # the heap overflow first), then both as the tests use them
    for name, flag, call, report in (
            ("asan", "-fsanitize=address", "c.heap(4)", "heap-buffer-overflow"),
            ("ubsan", "-fsanitize=undefined", "c.add(2147483647, 1)", "signed integer overflow"),
            ("both", "-fsanitize=address,undefined", "c.heap(4)", "runtime error")):
        lib = tmp_path / f"libcanary_{name}.so"
        flags = [f for f in GCC_SAN if not f.startswith("-fsanitize=")] + [flag]
        subprocess.run(["gcc", *flags, str(src), "-o", str(lib)], check=True)
        load = f"import ctypes; c = ctypes.CDLL({str(lib)!r}); "
        r = _run([sys.executable, "-c", load + "c.heap(1); c.add(1, 2)"], pre)
        assert r.returncode == 0, (name, r.stderr[-2000:])
        r = _run([sys.executable, "-c", load + call], pre)
        assert r.returncode != 0 and report in r.stderr, (name, r.stderr[-2000:])


def test_oracle_and_cpu_helpers_under_sanitizers(tmp_path):
    libs = _build_helpers(str(tmp_path))
    env = {"LD_PRELOAD": _gcc_runtime(), **libs}
    # the instrumented builds are the ones loaded
    check = ("import oracle, cpu_peel, bigraph_gen; oracle._load(); cpu_peel._load(); "
             "bigraph_gen._load(); maps = open('/proc/self/maps').read(); "
             f"assert all(p in maps for p in {sorted(libs.values())!r}), 'not loaded'; "
             "assert 'libasan' in maps and 'libubsan' in maps")
    r = _run([sys.executable, "-c", check], env)
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
              "tests/test_oracle_pins.py", "tests/test_cpu_peel.py"], env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_library_host_code_under_sanitizers(tmp_path):
    runtime = _clang_runtime()
    if runtime is None:
        pytest.skip("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    here = os.path.join(ROOT, "paper_2606_07148_amd")
    srcs = sorted(glob.glob(os.path.join(here, "csrc", "*.hip")))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(here, "csrc")]
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]

    def compile_one(pair):
        s, o = pair
        subprocess.run(["hipcc", "-c", *flags, s, "-o", o], check=True, capture_output=True)

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    lib = str(tmp_path / "libabcore.so")
    subprocess.run(["hipcc", "-shared", "--offload-arch=gfx950", "-fPIC", "-shared-libasan",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    *objs, "-o", lib], check=True, capture_output=True)
    env = {"LD_PRELOAD": runtime, "ABCORE_LIBRARY": lib}
    check = ("import paper_2606_07148_amd as p; p.load(); "
             f"assert {lib!r} in open('/proc/self/maps').read()")
    r = _run([sys.executable, "-c", check], env)
    assert r.returncode == 0, r.stderr[-3000:]
    # argument validation of every entry point and the batch planner (host
    # logic), which run without a GPU
    r = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
              "tests/test_abi_cpu.py", "tests/test_batch_plan.py"], env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
