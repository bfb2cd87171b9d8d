"""Run the gfx950 unit-throughput probe (LDS read/write widths, the hop kernel's update
pattern, FP32 and integer multiply, log2) that sets the roofline denominators.

    python -m paper_1407_5026_amd.probe

The probe is a standalone HIP program built by ``build.py`` next to the library; it prints
one line per measurement, rates per CU at 2.4 GHz."""
from __future__ import annotations

import os
import subprocess
import sys

from paper_1407_5026_amd.build import PROBE


def main() -> int:
    if not os.path.exists(PROBE):
        print(f"{PROBE} is not built; run python paper_1407_5026_amd/build.py", file=sys.stderr)
        return 2
    return subprocess.call([PROBE])


if __name__ == "__main__":
    sys.exit(main())
