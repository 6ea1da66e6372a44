"""Project NTSC palette, reduced to the 128-entry gray table the observation
path uses.

The paper does not give a palette (its frames are the console's 160x210
colour output, Section 3); the real console palette is not reproduced here.
This table is generated from a documented YIQ model and handed to both the CPU
oracle and the GPU library as plain input data:

* colour byte c -> index i = c >> 1 (bit 0 of a colour register is unused);
* hue = i >> 3 (0..15), luma = i & 7 (0..7);
* Y = luma / 7; hue 0 is achromatic, hue h >= 1 has phase (h - 1) * 24 degrees
  and amplitude 0.25 on the I/Q plane;
* RGB from the standard YIQ -> RGB matrix, clamped to [0, 1], scaled to 0..255
  and rounded;
* gray = (299 R + 587 G + 114 B + 500) // 1000.
"""

import math


def rgb_table():
    out = []
    for i in range(128):
        hue, luma = i >> 3, i & 7
        y = luma / 7.0
        if hue == 0:
            ci = cq = 0.0
        else:
            th = math.radians((hue - 1) * 24.0)
            ci, cq = 0.25 * math.cos(th), 0.25 * math.sin(th)
        r = y + 0.956 * ci + 0.621 * cq
        g = y - 0.272 * ci - 0.647 * cq
        b = y - 1.106 * ci + 1.703 * cq
        out.append(tuple(int(round(min(max(v, 0.0), 1.0) * 255)) for v in (r, g, b)))
    return out


def gray_table() -> bytes:
    return bytes((299 * r + 587 * g + 114 * b + 500) // 1000 for r, g, b in rgb_table())


GRAY = gray_table()
