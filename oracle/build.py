"""Compile the oracle's C source into ``oracle/liboracle.so`` (test
infrastructure; the device library never links it)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fsm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra",
                           "-Wno-unused-parameter", "-shared", "-fPIC",
                           SRC, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(out: str) -> str:
    """The same source built with AddressSanitizer and UndefinedBehavior-
    Sanitizer (host code only) into ``out``; a process that loads it must
    preload the ASan runtime (tests/test_oracle_sanitized.py)."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-std=c99", "-Wall", "-Wextra", "-Wno-unused-parameter",
                           "-shared", "-fPIC", SRC, "-o", out])
    return out


if __name__ == "__main__":
    print(build())
