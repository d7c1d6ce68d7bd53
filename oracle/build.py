"""Build the CPU oracle library (plain C, FP64, OpenMP over rows).

TEST INFRASTRUCTURE ONLY: the library this builds is loaded by ``tests/``,
``__graft_entry__.smoke()`` and the CPU leg of ``bench.py``, never by the
product path; ``__graft_entry__.build()`` compiles it so that the checker is
ready, which is not a use of it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "oracle.c")
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_sanitized(out_dir: str, verbose: bool = False) -> str:
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc's runtimes: preload the path of ``gcc -print-file-name=libasan.so``)."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-Wall", "-Wextra", "-o", out, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
