"""Build the serving-pool stress driver against the fake HIP backend, for the
CPU under AddressSanitizer ('address') or ThreadSanitizer ('thread').
Host code only: gbees.cpp, fake_hip.cpp and pool_stress.cpp are compiled for
the host (no device code) and linked without the HIP runtime."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2508_13986_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


def build(kind="address", out_dir=None):
    out_dir = out_dir or os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    srcs = [os.path.join(CSRC, "gbees.cpp"), os.path.join(HERE, "fake_hip.cpp"), os.path.join(HERE, "pool_stress.cpp")]
    objs = []
    for src in srcs:
        obj = os.path.join(out_dir, f"{os.path.basename(src)}.{kind}.o")
        subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
                        "-fno-omit-frame-pointer", "-Xarch_host", f"-fsanitize={kind}", "-w",
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj], check=True)
        objs.append(obj)
    exe = os.path.join(out_dir, f"pool_stress_{kind}")
    subprocess.run([CLANG, f"-fsanitize={kind}", "-o", exe, *objs, "-lpthread"], check=True)
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else "address"))
