"""Build the test-only host harness of the coefficient routines (libcoefhost.so)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
LIB = os.path.join(HERE, "libcoefhost.so")


def build():
    from paper_1006_0663_amd import build as pb
    cmd = [pb.HIPCC] + pb.FLAGS + ["-shared", "-o", LIB + ".tmp", os.path.join(HERE, "coef_host.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr[-4000:])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
