"""Write closed_forms.json: PSDF values derived by hand from the paper's
definitions for a rectangle footprint against single segments.

Nothing here calls the oracle or the HIP path; every expected value is a
closed-form expression evaluated in float64 on the float32-rounded inputs.
Run:  python tests/golden/make_closed_forms.py
"""
import json
import math
import os

import numpy as np

f = lambda x: float(np.float32(x))  # noqa: E731  (inputs are float32)

A, B = f(0.3), f(0.2)          # half extents of the 0.6 x 0.4 m rectangle
FP = [[-A, -B], [A, -B], [A, B], [-A, B]]
ETA = 1000.0
cases = []

# CF1 - face contact (Sec. IV-B pools; Sec. IV-A transform).  Segment y = y0
# above the robot at heading th: the nearest robot point is the rotated corner
# (a, b), whose height is a sin th + b cos th.
y0, th = f(0.5), f(0.1)
cases.append(dict(
    name="CF1_face", cite="Sec. IV-A eq. for A~; Sec. IV-B eqs. for u, t, d, d_sep",
    footprint=FP, pose=[0.0, 0.0, th], edges=[[f(-1), y0, f(1), y0]], eta=ETA,
    phi=y0 - A * math.sin(th) - B * math.cos(th),
    grad=[0.0, -1.0, -(A * math.cos(th) - B * math.sin(th))], edge=0, pen=0,
    derivation="phi = y0 - a sin(th) - b cos(th); dphi/dy = -1; dphi/dth = -(a cos th - b sin th)"))

# CF2 - vertex-vertex contact: corner c = (a, b), segment endpoint o = (0.6, 0.6).
o = (f(0.6), f(0.6))
dx, dy = o[0] - A, o[1] - B
r = math.hypot(dx, dy)
nx, ny = dx / r, dy / r
cases.append(dict(
    name="CF2_vertex_vertex", cite="Sec. IV-B eqs. for d_v, d_e, d_sep",
    footprint=FP, pose=[0.0, 0.0, 0.0], edges=[[o[0], o[1], f(0.6), f(2.0)]], eta=ETA,
    phi=r, grad=[-nx, -ny, nx * B - ny * A], edge=0, pen=0,
    derivation="phi = |o - c|; grad_p = -(o-c)/|o-c|; dphi/dth = -n.(dc/dth), dc/dth = (-b, a)"))

# CF3 - penetration by a segment at y = y0 inside the robot.  Axes: +-y robot
# normals and the segment normal overlap by b - y0; the +-x robot normals by 1 + a.
y0 = f(0.05)
dy_, dx_ = B - y0, 1.0 + A
phi = -dy_ + math.log(3.0 + 2.0 * math.exp(-ETA * (dx_ - dy_))) / ETA
cases.append(dict(
    name="CF3_penetration_soft", cite="Sec. IV-C eqs. for delta, separated, soft-min depth; Sec. IV-D",
    footprint=FP, pose=[0.0, 0.0, 0.0], edges=[[f(-1), y0, f(1), y0]], eta=ETA,
    phi=phi, grad=[0.0, -1.0, None], edge=0, pen=1,
    derivation="phi = -(b - y0) + ln(3 + 2 exp(-eta((1 + a) - (b - y0))))/eta"))
cases.append(dict(
    name="CF3_penetration_hard", cite="Sec. IV-C (eta -> inf limit of the soft-min)",
    footprint=FP, pose=[0.0, 0.0, 0.0], edges=[[f(-1), y0, f(1), y0]], eta=math.inf,
    phi=-dy_, grad=[0.0, -1.0, None], edge=0, pen=1, derivation="phi = -(b - y0)"))

# CF4a - touching a parallel segment at y = b: three axes with zero overlap,
# two with 1 + a.  The strict test delta < -eps_sat is false, so the
# non-separated branch applies and the soft-min gives +ln(3)/eta.
cases.append(dict(
    name="CF4a_touch_parallel_soft", cite="Sec. IV-C separated test and soft-min; Sec. IV-D",
    footprint=FP, pose=[0.0, 0.0, 0.0], edges=[[f(-1), B, f(1), B]], eta=ETA,
    phi=math.log(3.0 + 2.0 * math.exp(-ETA * (1.0 + A))) / ETA, grad=None, edge=0, pen=1,
    derivation="phi = ln(3 + 2 exp(-eta (1 + a)))/eta"))
cases.append(dict(
    name="CF4a_touch_parallel_hard", cite="Sec. III-B (sd = 0 at contact)",
    footprint=FP, pose=[0.0, 0.0, 0.0], edges=[[f(-1), B, f(1), B]], eta=math.inf,
    phi=0.0, grad=None, edge=0, pen=1, derivation="phi = 0"))

# CF4b - segment on the supporting line x + y = a + b through corner (a, b);
# every other axis overlaps by 0.5, so phi ~ e^{-500}/eta ~ 0 (float32 inputs
# leave a residual of order 1e-8).
cases.append(dict(
    name="CF4b_touch_corner", cite="Sec. III-B (sd = 0 at contact); Sec. IV-C",
    footprint=FP, pose=[0.0, 0.0, 0.0], edges=[[f(0.8), f(-0.3), f(-0.2), f(0.7)]], eta=ETA,
    phi=0.0, phi_tol=1e-6, grad=None, edge=0, pen=None, derivation="phi ~ 0"))

out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")
with open(out, "w") as fh:
    json.dump(dict(source="closed forms derived from the PSDF definitions (Sec. III-B, IV-A..IV-D)",
                   eps=1e-12, eps_sat=1e-6, cases=cases), fh, indent=1,
              default=lambda x: None)
print("wrote", out)
