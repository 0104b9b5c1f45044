"""Readers of the fixture files under tests/golden/ (values the paper prints, with their citations
in each file's header)."""

import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def table1():
    """Sec. 5.2, Table 1: {gate name: (qubits, optimal T-count)}."""
    rows = {}
    with open(os.path.join(GOLDEN, "table1_optimal_tcount.txt")) as f:
        for line in f:
            fields = line.split("#", 1)[0].split()
            if fields:
                rows[fields[0]] = (int(fields[1]), int(fields[2]))
    return rows
