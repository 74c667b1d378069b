"""Run the oracle pins against one compiled oracle copy (used by
test_oracle_mutants in a child process, so that a planted mistake that
crashes cannot take the test runner down).  Exit status 0 = every pin held."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from tests import pins  # noqa: E402


def main(path):
    o = oracle.Oracle(path)
    pin_set = pins.ALL_SGEMM_PINS + pins.ALL_DGEMM_PINS + pins.ALL_LU_PINS + [
        lambda o: pins.pin_bf16_rne_vs_torch(o, count=1 << 16),
        lambda o: pins.pin_bf16x3_exhaustive(o, 0x3F800000, 0x3F800000 + (1 << 22)),
        pins.pin_bf16x3_method,
    ]
    failed = []
    for pin in pin_set:
        try:
            pin(o)
        except (AssertionError, ValueError):
            failed.append(getattr(pin, "__name__", "lambda"))
    print("failed pins:", failed)
    return 1 if failed else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
