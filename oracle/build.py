"""Build liboracle.so from abm_oracle.c with the host C compiler (test infrastructure).

build()        the library the tests load (portable flags, next to the source).
build_native() the same source with -O3 -march=native into a directory of the
               caller's choosing, for timing the oracle on the host it runs on
               (built there, since -march=native code may not run elsewhere).
"""
import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abm_oracle.c")
_WARN = ["-std=c11", "-Wall", "-Wextra", "-Werror", "-shared", "-fPIC", "-fvisibility=hidden"]


def _compile(out: str, opt, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = ["gcc", *opt, *_WARN, "-o", tmp, _SRC]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    return _compile(os.path.join(_HERE, "liboracle.so"), ["-O2"], verbose)


def build_native(out_dir: str, verbose: bool = False) -> str:
    os.makedirs(out_dir, exist_ok=True)
    return _compile(os.path.join(out_dir, "liboracle_native.so"), ["-O3", "-march=native"],
                    verbose)


if __name__ == "__main__":
    print(build(verbose=True))
