"""Write near_contact_figure.txt from the near-contact criterion figure.

The figure of the section "The no-coalescence.h algorithm" (the sketch of
the near-contact criterion, both panels) is drawn from explicit rules: a
grid cell whose lower-left corner (col, row) lies strictly closer than r to
a given point belongs to a region. This script evaluates those rules; it
uses no part of the method. Characters: '1', '2' = the two tags of tracer i,
'j' = tracer j, '.' = empty.

Left panel: 20 x 10 cells; tag 1 within 4 of (4.356, 2.65), tag 2 within
3.5 of (15, 6.2) (both tracer i); tracer j within 2.5 of (15.62, 1.5).
Right panel: 10 x 10 cells; one tracer-i region made of four discs of
radius 3.5 around (0,2), (7,2), (5,0) and (0,9), all drawn with tag 1.
"""
import math
import os


def panel(ncol, nrow, shapes):
    g = [["." for _ in range(ncol)] for _ in range(nrow)]
    for (cx, cy, r, ch) in shapes:
        for row in range(nrow):
            for col in range(ncol):
                if math.hypot(col - cx, row - cy) < r:
                    if ch == "j" and g[row][col] != ".":
                        g[row][col] = "*"  # tracer i and tracer j both occupy the cell
                    elif g[row][col] == "j" and ch != "j":
                        g[row][col] = "*"
                    else:
                        g[row][col] = ch
    return ["".join(r) for r in g]


left = panel(20, 10, [(4.356, 2.65, 4.0, "1"), (15, 6.2, 3.5, "2"), (15.62, 1.5, 2.5, "j")])
right = panel(10, 10, [(0, 2, 3.5, "1"), (7, 2, 3.5, "1"), (5, 0, 3.5, "1"), (0, 9, 3.5, "1")])

out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "near_contact_figure.txt")
with open(out, "w") as f:
    f.write("# Near-contact criterion figure, section 'The no-coalescence.h algorithm'.\n")
    f.write("# Rows listed from row 0 (bottom of the figure) upwards; '*' = tracer i tag 2 and tracer j overlap.\n")
    f.write("# Expected (Step 4): left, the drop of tag 2 moves to a new tracer n not in {i, j};\n")
    f.write("# right, one region close to itself: no move (Step 3).\n")
    f.write("[left]\n")
    f.write("\n".join(left) + "\n")
    f.write("[right]\n")
    f.write("\n".join(right) + "\n")
print(out)
