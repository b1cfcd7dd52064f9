"""Dependency cones of the colour phases (test helper; no method arithmetic).

In a sweep, a cell of colour phase q reads the disks its eight neighbours of
earlier phases have moved (Sec. 3.4, steps 4-6).  The cone of a cell is the
cell together with its earlier-phase neighbours, recursively: replaying only
the cells of a cone from the positions at the start of the sweep reproduces
the cell exactly.
"""


def phase_of_cell(C, perm, cell):
    """Phase (0-3) in which `cell` runs, for the colour order perm of the sweep."""
    colour = (cell % C & 1) | ((cell // C & 1) << 1)
    return [int(v) for v in perm].index(colour)


def dependency_cone(C, perm, cell):
    """Set of cells whose phase work `cell` depends on (itself included)."""
    out = {int(cell)}
    front = [int(cell)]
    while front:
        c = front.pop()
        q = phase_of_cell(C, perm, c)
        cx, cy = c % C, c // C
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == 0 and dy == 0:
                    continue
                nc = ((cy + dy) % C) * C + (cx + dx) % C
                if nc not in out and phase_of_cell(C, perm, nc) < q:
                    out.add(nc)
                    front.append(nc)
    return out
