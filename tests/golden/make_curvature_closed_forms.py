"""Writes curvature_closed_forms.json: closed-form curvatures of analytic graphs.

Every number comes from a textbook closed form (cited per case); nothing here
calls the oracle or the GPU path.  "mc" is the divergence form of Table 1
(= 2H), "gc" is det(Hess u) / (1 + |grad u|^2)^2 (= K).
"""
import json
import math
import os

cases = []
R = 2.0
cases.append(dict(surface="sphere", params={"R": R}, x=0.3, y=-0.4, mc=-2.0 / R, gc=1.0 / R**2,
    source="upper hemisphere of radius R: 2H = -2/R, K = 1/R^2 (do Carmo, Differential Geometry of Curves and Surfaces, Sec. 3-3)"))
cases.append(dict(surface="cylinder", params={"R": R}, x=0.5, y=0.7, mc=-1.0 / R, gc=0.0,
    source="z = sqrt(R^2 - x^2): principal curvatures -1/R and 0, so 2H = -1/R, K = 0 (do Carmo Sec. 3-3)"))
x, y = 1.0, 0.5
cases.append(dict(surface="helicoid", params={}, x=x, y=y, mc=0.0, gc=-1.0 / (1.0 + x * x + y * y) ** 2,
    source="z = atan(y/x): helicoid, a minimal surface (H = 0) with K = -1/(1 + x^2 + y^2)^2 (do Carmo Sec. 3-5)"))
x, y = 0.3, 0.2
q = 1.0 + x * x + y * y
cases.append(dict(surface="saddle", params={}, x=x, y=y, mc=-2.0 * x * y / q ** 1.5, gc=-1.0 / q ** 2,
    source="z = x y: 2H = -2 x y / (1 + x^2 + y^2)^(3/2), K = -1/(1 + x^2 + y^2)^2 (do Carmo Sec. 3-3)"))
cases.append(dict(surface="scherk_rotated", params={"angle": math.pi / 4}, x=0.2, y=0.1, mc=0.0, gc=None,
    source="z = log(cos(Y)/cos(X)), (X, Y) = the plane rotated by 45 degrees: Scherk's first surface, minimal, H = 0 (do Carmo Sec. 3-5); the rotation makes u_xy non-zero"))
cases.append(dict(surface="paraboloid", params={"a": 1.5, "b": -0.5}, x=0.0, y=0.0, mc=1.0, gc=-0.75,
    source="z = (a x^2 + b y^2)/2 at the origin: principal curvatures a and b, so 2H = a + b, K = a b"))

doc = {"description": "Closed-form curvatures of analytic graphs, used to pin the 3x3 finite-difference "
       "curvature of Table 1 (mean curvature in divergence form, i.e. 2H; Gaussian curvature K). "
       "Values are from the closed forms cited per case, not from any implementation.",
       "cases": cases}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "curvature_closed_forms.json"), "w") as fh:
    json.dump(doc, fh, indent=1)
