"""Progress lines for long GPU tests: stderr plus gpurun_out/progress.log when present."""

import os
import sys
import time

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_T0 = time.time()


def say(*parts):
    msg = f"[{time.time() - _T0:7.1f}s] " + " ".join(str(p) for p in parts)
    print(msg, file=sys.stderr, flush=True)
    out = os.path.join(_ROOT, "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "progress.log"), "a") as f:
            f.write(msg + "\n")
