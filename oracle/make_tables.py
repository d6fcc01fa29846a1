"""Write the oracle's FC(Gram) table file (calls only ``oracle/``).

Usage:  python -m oracle.make_tables      (about half a minute; mpmath at 64 digits)
"""
from __future__ import annotations

import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import fcgram  # noqa: E402


def main() -> None:
    tabs, _ = fcgram.build()
    os.makedirs(fcgram.TABLE_DIR, exist_ok=True)
    path = fcgram.default_table_path(tabs.params["d"], tabs.params["C"])
    fcgram.write_table(tabs, path)
    print("wrote", path, "residuals", tabs.residuals)


if __name__ == "__main__":
    main()
