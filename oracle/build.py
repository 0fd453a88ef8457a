"""Build the CPU oracle (test infrastructure only) into oracle/liboracle.so with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")
SOURCES = ["orc_graph.c", "orc_pattern.c", "orc_ns.c", "orc_gs.c", "orc_learned.c"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(SO):
        tmp = SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
               "-Wall", "-Wno-unused-function"]
        cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build())
