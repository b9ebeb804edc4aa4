"""Build the C consumer of the library's C ABI (tests/native/abi_roundtrip.c)
with gcc against include/pyrit.h, libpyrit.so and the HIP runtime."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1709_00178_amd")
SRC = os.path.join(HERE, "abi_roundtrip.c")
EXE = os.path.join(HERE, "abi_roundtrip")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_abi_roundtrip() -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}", SRC,
           f"-L{PKG}", "-lpyrit", f"-L{ROCM}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1709_00178_amd", f"-Wl,-rpath,{ROCM}/lib",
           "-o", EXE + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build_abi_roundtrip())
