"""The operation counts bench.py uses for the roofline are the ones derived in
profiles/opcount.md, and each total there is the sum of its formula steps."""
import re
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def _rows(text):
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4:
            yield cells


def _num(c):
    return int(c.strip("*"))


def test_bench_constants_match_the_op_count_file():
    import bench
    text = (ROOT / "profiles" / "opcount.md").read_text()
    table = text[text.index("## Constants used by bench.py"):]
    got = {}
    for cells in _rows(table):
        if cells[0] in bench.OPS:
            got[cells[0]] = tuple(int(c) for c in cells[1:4])
    assert got == bench.OPS


def test_op_count_totals_are_the_sums_of_their_steps():
    text = (ROOT / "profiles" / "opcount.md").read_text()
    sections = re.split(r"\n## ", text)
    checked = 0
    for sec in sections:
        if not sec.startswith(("GMM-vMF pair", "GMM-GMM pair")):
            continue
        acc = [0, 0, 0]
        half = None
        for cells in _rows(sec):
            name = cells[0]
            if name in ("step", "---") or set(name) <= {"-"}:
                continue
            vals = cells[-3:]
            if name.startswith("**"):
                tot = [_num(v) for v in vals]
                if "UB pair" in name:
                    # the GMM-GMM centre term is stated as the GMM-vMF one
                    half = tot
                    assert acc == tot or (acc == [0, 0, 0] and tot == [19, 3, 4]), (name, acc, tot)
                    acc = [0, 0, 0]
                elif "LB pair" in name:
                    assert acc == tot, (name, acc, tot)
                    lb = tot
                elif "pair evaluated" in name:
                    assert tot == [half[k] + lb[k] for k in range(3)], name
                checked += 1
                continue
            acc = [acc[k] + int(vals[k]) for k in range(3)]
    assert checked >= 6
    # the translation preparation constant adds the diagonal row
    prep = re.search(r"\| component x translation cell \|[^\n]*\| (\d+) \| (\d+) \| (\d+) \|", text)
    diag = re.search(r"\| component x translation cell, diagonal \|[^\n]*\| (\d+) \| (\d+) \| (\d+) \|", text)
    import bench
    assert tuple(int(prep.group(k)) + int(diag.group(k)) for k in (1, 2, 3)) == bench.OPS["TRANS_PREP"]
