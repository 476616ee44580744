"""Builds tests/c_abi_client (a plain C99 program against include/impconv.h
and libimpconv.so) with gcc; -pedantic -Werror checks that the public
header is valid C on its own."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c_abi_client.c")
BIN = os.path.join(HERE, "c_abi_client")
LIBDIR = os.path.join(ROOT, "paper_1008_1366_amd")
HEADER = os.path.join(ROOT, "include", "impconv.h")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command():
    return ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-pedantic", "-Werror",
            "-isystem", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
            SRC, "-o", BIN, "-L", LIBDIR, "-limpconv", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
            "-Wl,-rpath," + LIBDIR, "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(p) for p in (SRC, HEADER, os.path.join(LIBDIR, "libimpconv.so")))
    if force or not os.path.exists(BIN) or os.path.getmtime(BIN) < newest:
        subprocess.run(command(), check=True, capture_output=True, text=True)
    return BIN
