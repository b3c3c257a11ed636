"""The library's plan and scheduler code (plan.cpp) built for the host against a stand-in HIP
runtime (tests/hostsim): kernels are stubs that record their launches, device memory is host
memory, so the control flow runs on the CPU under AddressSanitizer and UBSan — workspace set-up
and release, the pass schedule, the panel order of the streamed sources (Section 4.2) and their
callbacks, and the error paths under injected allocation, copy and launch failures."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "hostsim")
CSRC = os.path.join(ROOT, "paper_1007_5510_amd", "csrc")
CXX = "/opt/rocm/llvm/bin/clang++"


def launcher_stubs(kernels_h: str) -> str:
    """One recording stub per `hipError_t launch_*(...)` declaration of the kernel interface."""
    text = re.sub(r"//[^\n]*", "", open(kernels_h).read())
    out = ["// generated from kernels.h by tests/test_host_runtime.py", "#include <hip/hip_runtime.h>",
           '#include "hostsim.h"', f'#include "{kernels_h}"', "namespace rpca {"]
    for m in re.finditer(r"hipError_t\s+(launch_\w+)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        name, params = m.group(1), m.group(2)
        params = re.sub(r"\s*=\s*[^,]+", "", params)  # default arguments stay in the declaration
        out.append(f"hipError_t {name}({params}) {{ return (hipError_t)hostsim::launch(\"{name}\"); }}")
    out.append("}  // namespace rpca")
    return "\n".join(out) + "\n"


@pytest.fixture(scope="module")
def hostsim_binary(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("host clang++ not available")
    d = tmp_path_factory.mktemp("hostsim")
    stubs = d / "stubs.cpp"
    stubs.write_text(launcher_stubs(os.path.join(CSRC, "kernels.h")))
    exe = d / "hostsim"
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", SIM, "-I", SIM + "/..",
           os.path.join(CSRC, "plan.cpp"), os.path.join(SIM, "hostsim_rt.cpp"), os.path.join(SIM, "hostsim_extra.cpp"),
           os.path.join(SIM, "hostsim_main.cpp"), str(stubs), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def test_plan_runtime_on_host_under_sanitizers(hostsim_binary):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(hostsim_binary)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-6000:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "ALL PASSED" in r.stdout
    passed = [l for l in r.stdout.splitlines() if l.startswith("PASS ")]
    assert len(passed) == 17
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


def test_every_launcher_is_stubbed():
    """The stub generator sees every launcher the kernel interface declares."""
    text = re.sub(r"//[^\n]*", "", open(os.path.join(CSRC, "kernels.h")).read())
    declared = set(re.findall(r"hipError_t\s+(launch_\w+)\s*\(", text))
    generated = set(re.findall(r"hipError_t (launch_\w+)\(", launcher_stubs(os.path.join(CSRC, "kernels.h"))))
    assert declared == generated and len(declared) > 50
