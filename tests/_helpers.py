"""Shared helpers for the tests (no method arithmetic here)."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lalm.h")
LIB = os.path.join(ROOT, "paper_1402_4381_amd", "liblalm.so")


def ensure_built():
    """Build the HIP library only when nothing is built yet."""
    if not os.path.exists(LIB):
        subprocess.check_call([sys.executable, "-m", "paper_1402_4381_amd.build"], cwd=ROOT)
    return LIB


def header_functions():
    """Every call declared (LALM_API) in include/*.h."""
    import glob
    text = "".join(open(p).read() for p in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    return sorted(set(re.findall(r"LALM_API\s+[\w\s\*]*?\b(lalm_\w+)\s*\(", text)))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
