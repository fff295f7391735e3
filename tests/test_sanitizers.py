"""The oracle and the host side of liblf under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

  - the oracle (plain C) built with gcc -fsanitize=address,undefined runs its
    pins (tests/test_oracle_pins.py) with no report;
  - liblf built with the sanitizers on its host code only (-Xarch_host; the
    gfx950 code is built as usual) runs the ABI and request-loop tests that need
    no GPU (tests/test_abi.py, tests/test_server_cpu.py): argument checks,
    workspace arithmetic, the server's queues, arena and failure paths.

Each runs in a child process with the sanitizer runtime preloaded.  Skipped
when the process already has a preload (it is never replaced) or a compiler is
missing."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _no_preload():
    if os.environ.get("LD_PRELOAD"):
        return False
    p = "/etc/ld.so.preload"
    return not (os.path.exists(p) and os.path.getsize(p) > 0)


pytestmark = pytest.mark.skipif(not _no_preload(), reason="a preload is configured")

_ENV = dict(ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
            UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _child(code, preload, timeout):
    env = dict(os.environ, LD_PRELOAD=preload, **_ENV)
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=timeout)
    return res.returncode, res.stdout[-3000:] + res.stderr[-3000:]


def test_oracle_pins_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    lib = str(tmp_path / "liblfo_san.so")
    subprocess.check_call([gcc, "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "lfo.c"), "-lm"])
    rt = [subprocess.check_output([gcc, f"-print-file-name={n}"], text=True).strip()
          for n in ("libasan.so", "libubsan.so")]
    code = ("import sys, oracle, pytest\n"
            f"oracle._LIB_PATH = {lib!r}\n"
            "oracle._lib = None\n"
            "oracle.build = lambda *a, **k: oracle._LIB_PATH\n"
            "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', "
            "'tests/test_oracle_pins.py']))\n")
    rc, out = _child(code, " ".join(rt), 900)
    assert rc == 0, out


@pytest.mark.slow
def test_host_library_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/lib/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("no hipcc")
    from paper_1907_13449_amd import build as b
    san = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    for src in b.sources():
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, *b.compile_flags(), *san, "-c", "-o", obj, src],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-2000:]
    lib = str(tmp_path / "liblf_san.so")
    subprocess.check_call([hipcc, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", "-Xarch_host",
                           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", lib,
                           *objs], stderr=subprocess.DEVNULL)
    rt = subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                 text=True).strip()
    # the binding loaded against the sanitized library, under its usual module name
    old, new = 'LIB_PATH = os.path.join(_HERE, "liblf.so")', f"LIB_PATH = {lib!r}"
    code = ("import sys, types\n"
            "import paper_1907_13449_amd as pkg\n"
            "src = open('paper_1907_13449_amd/lf.py').read()\n"
            f"assert {old!r} in src\n"
            f"src = src.replace({old!r}, {new!r})\n"
            "m = types.ModuleType('paper_1907_13449_amd.lf')\n"
            "m.__file__ = 'paper_1907_13449_amd/lf.py'\n"
            "m.__package__ = 'paper_1907_13449_amd'\n"
            "sys.modules['paper_1907_13449_amd.lf'] = m\n"
            "exec(compile(src, m.__file__, 'exec'), m.__dict__)\n"
            "pkg.lf = m\n"
            f"assert m.lib._name == {lib!r}\n"
            "import pytest\n"
            "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu', "
            "'tests/test_abi.py', 'tests/test_server_cpu.py']))\n")
    rc, out = _child(code, rt, 900)
    assert rc == 0, out
