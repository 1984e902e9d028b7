"""Runs the oracle pins against one compiled oracle variant in a process of
its own (a planted mistake may crash the process; that counts as caught).
Usage: python mutant_runner.py <path-to-variant.so>.  Exit status 0 means
every pin passed (the mutant was NOT caught); 1 means a pin failed."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle as O  # noqa: E402
import oracle_pins as P  # noqa: E402


def main(path: str) -> int:
    with O.use_library(path):
        for check in P.ALL_CHECKS:
            try:
                check()
            except Exception as e:  # noqa: BLE001
                print("caught by", check.__name__, type(e).__name__)
                return 1
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
