"""The task numbering of the dataflow solves (flow_tasks_kernel), restated
here: for every block count R, each task of the blocked
schedule (Section "Data Locality": per round, the diagonal block, its block
row and column, then the remaining blocks) appears exactly once, and every
task's operands -- its own block's previous round, the closed diagonal
block or the two panels of its round -- come from strictly smaller numbers.
That order is what lets a launch complete however few of its workgroups
are resident: a workgroup only ever waits for numbers that running
workgroups hold.  (A model of the numbering, checked on the CPU; the GPU
parity tests run the kernel itself.)"""
import pytest


def decode(R):
    """[(number, task)] with task ('P1',) for round 0's closure of block
    (0, 0), else (r, i, j): round r's product on block (i, j) (block (r+1,
    r+1) includes its closure for round r+1)."""
    m = R - 1
    if R == 1:
        return [(0, ("P1",))]
    per_round = 2 * (R - 1) + 1 + 2 * (R - 2) + (R - 2) ** 2
    last = 2 * (R - 1) + (R - 1) ** 2
    assert per_round == last == (R - 1) * (R + 1)  # the kernel's count per round
    total = 1 + (R - 1) * per_round + last
    out = [(0, ("P1",))]
    for t in range(1, total):
        t1 = t - 1
        ahead = t1 < (R - 1) * per_round
        r = t1 // per_round if ahead else R - 1
        u = t1 % per_round if ahead else t1 - (R - 1) * per_round
        if u < 2 * m:
            row = u < m
            q = u if row else u - m
            q += q >= r
            out.append((t, (r, r, q) if row else (r, q, r)))
            continue
        u -= 2 * m
        if ahead:
            w = m - 1
            skip2 = lambda q: q + (2 if q >= r else 0)  # noqa: E731
            if u == 0:
                out.append((t, (r, r + 1, r + 1)))
            elif u - 1 < 2 * w:
                x = skip2((u - 1) % w)
                out.append((t, (r, r + 1, x) if u - 1 < w else (r, x, r + 1)))
            else:
                a = u - 1 - 2 * w
                out.append((t, (r, skip2(a // w), skip2(a % w))))
        else:
            out.append((t, (r, u // m + (u // m >= r), u % m + (u % m >= r))))
    return out


def test_task_numbering_complete_and_ordered():
    for R in list(range(1, 34)) + [48, 64, 96]:
        seen = {}
        for t, task in decode(R):
            assert t == len(seen), (R, t)  # numbers 0, 1, 2, ... one task each
            assert task not in seen, (R, task)
            seen[task] = t
        expect = {("P1",)} | {(r, i, j) for r in range(R) for i in range(R) for j in range(R)
                               if not (i == r and j == r)}
        assert set(seen) == expect, R

        def number(r, i, j):
            if i == r and j == r:  # closed block r: round r-1's block (r, r), or the first task
                return seen[("P1",)] if r == 0 else seen[(r - 1, r, r)]
            return seen[(r, i, j)]

        for task, t in seen.items():
            if task == ("P1",):
                continue
            r, i, j = task
            deps = [number(r - 1, i, j)] if r > 0 else []
            if i == r or j == r:
                deps.append(number(r, r, r))
            else:
                deps += [number(r, i, r), number(r, r, j)]
            assert all(d < t for d in deps), (R, task, t, deps)
