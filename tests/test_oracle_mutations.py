"""The oracle's pins have teeth: each planted mistake fails at least one pin.

Every mutant is a one-spot text edit of a copy of the oracle's C source,
compiled with gcc into a temporary directory and swapped in for the real
oracle while the pin tests of ``test_oracle_pins`` run against it.  All of
this happens on the CPU.
"""
import inspect
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "fbp_oracle.c")

# (name, text to find, replacement); only the first occurrence is edited, which for the
# shared backprojection/splat expressions is the backprojector.
MUTANTS = [
    ("centre tap halved", "return 1.0 / (4.0 * dt * dt);", "return 1.0 / (8.0 * dt * dt);"),
    ("odd tap sign", "return -1.0 / (kPi * kPi * dd * dd * dt * dt);",
     "return 1.0 / (kPi * kPi * dd * dd * dt * dt);"),
    ("odd tap pi instead of pi^2", "return -1.0 / (kPi * kPi * dd * dd * dt * dt);",
     "return -1.0 / (kPi * dd * dd * dt * dt);"),
    ("even taps kept", "if (d % 2 == 0) return 0.0;", "if (d % 2 == 0) return -1.0 / (kPi * kPi * (double)d * (double)d * dt * dt);"),
    ("filter output missing dt", "q[n] = dt * acc;", "q[n] = acc;"),
    ("circular convolution", "ramlak((int64_t)n - m, dt)", "ramlak(((int64_t)n - m + D) % D, dt)"),
    ("filter kernel truncated", "for (int32_t m = 0; m < D; ++m) acc",
     "for (int32_t m = (n > 8 ? n - 8 : 0); m < (n + 9 < D ? n + 9 : D); ++m) acc"),
    ("x and y swapped", "(x * cs[2 * k] + y * cs[2 * k + 1])", "(y * cs[2 * k] + x * cs[2 * k + 1])"),
    ("sin sign flipped", "(x * cs[2 * k] + y * cs[2 * k + 1])", "(x * cs[2 * k] - y * cs[2 * k + 1])"),
    ("truncate instead of floor", "const double fi = floor(u);", "const double fi = trunc(u);"),
    ("detector centre off by half a bin", "const double centre_det = 0.5 * (double)(D - 1);",
     "const double centre_det = 0.5 * (double)D;"),
    ("pixel centre off by half a pixel", "const double centre_pix = 0.5 * (double)(N - 1);",
     "const double centre_pix = 0.5 * (double)N;"),
    ("no pi/K weight", "const double weight = kPi / (double)K;", "const double weight = 1.0 / (double)K;"),
    ("interpolation weights swapped", "(1.0 - alpha) * qtilde(q, D, i) + alpha * qtilde(q, D, i + 1)",
     "alpha * qtilde(q, D, i) + (1.0 - alpha) * qtilde(q, D, i + 1)"),
    ("edge clamped instead of zero", "return (i >= 0 && i < D) ? q[i] : 0.0;",
     "return q[i < 0 ? 0 : (i >= D ? D - 1 : i)];"),
    ("u not divided by dt", "y * cs[2 * k + 1]) / dt + centre_det", "y * cs[2 * k + 1]) + centre_det"),
    ("nearest neighbour", "const double alpha = u - fi;", "const double alpha = (u - fi) < 0.5 ? 0.0 : 1.0;"),
    ("last angle dropped", "for (int32_t k = 0; k < K; ++k) {\n                const double u",
     "for (int32_t k = 0; k < K - 1; ++k) {\n                const double u"),
    ("Shepp-Logan 4d^2+1", "(4.0 * dd * dd - 1.0)", "(4.0 * dd * dd + 1.0)"),
    ("Shepp-Logan sign", "return -2.0 / (kPi * kPi", "return 2.0 / (kPi * kPi"),
    ("Hann centre weight", "0.5 * ramlak(d, dt) + 0.25", "0.25 * ramlak(d, dt) + 0.25"),
    ("Hann one-sided", "(ramlak(d - 1, dt) + ramlak(d + 1, dt))", "(ramlak(d - 1, dt) + ramlak(d - 1, dt))"),
    ("weights without the half", "w[order[i]] = 0.5 * (next - prev);", "w[order[i]] = (next - prev);"),
    ("weights without wrap-around", "a[order[K - 1]] - kPi", "a[order[0]]"),
    ("weights not reduced to the half-turn", "double t = fmod(angles[k], kPi);", "double t = angles[k];"),
    ("weighted backprojection ignores weights", "acc += weights[k] * (", "acc += (kPi / (double)K) * ("),
    ("fan filter without the half", "acc += 0.5 * filter_tap(kind, (int64_t)n - m, ds)",
     "acc += filter_tap(kind, (int64_t)n - m, ds)"),
    ("fan pre-weight squared", "pw[m] = R / sqrt(R * R + s * s);", "pw[m] = R * R / (R * R + s * s);"),
    ("fan pre-weight missing", "pw[m] = R / sqrt(R * R + s * s);", "pw[m] = 1.0;"),
    ("fan magnification to the first power", "acc += wk * (R / L) * (R / L) * (", "acc += wk * (R / L) * ("),
    ("fan detector axis reversed", "const double sx = R * (-x * sb + y * cb) / L;",
     "const double sx = R * (x * sb - y * cb) / L;"),
    ("fan depth sign", "const double L = R - (x * cb + y * sb);", "const double L = R + (x * cb + y * sb);"),
    ("fan weight pi/K", "const double wk = 2.0 * kPi / (double)K;", "const double wk = kPi / (double)K;"),
    ("fan coordinate not divided by ds", "const double u = sx / ds + centre_det;", "const double u = sx + centre_det;"),
    ("cone pre-weight without the row", "sqrt(R * R + sm * sm + zj * zj)", "sqrt(R * R + sm * sm)"),
    ("cone filter without the half", "acc += 0.5 * filter_tap(kind, (int64_t)n - m, du)",
     "acc += filter_tap(kind, (int64_t)n - m, du)"),
    ("cone row not magnified", "const double v = R * z / L / dv + cv;", "const double v = z / dv + cv;"),
    ("cone row sign", "const double v = R * z / L / dv + cv;", "const double v = -R * z / L / dv + cv;"),
    ("cone bilinear corner", "a * bb * qcone(q, Dv, Du, i + 1, j + 1)", "a * bb * qcone(q, Dv, Du, i + 1, j)"),
    ("cone detector transposed", "q[j * (int64_t)Du + i]", "q[i * (int64_t)Dv + j]"),
    ("cone weight pi/K", "centre_z = 0.5 * (double)(Nz - 1);\n    const double weight = 2.0 * kPi / (double)K;",
     "centre_z = 0.5 * (double)(Nz - 1);\n    const double weight = kPi / (double)K;"),
    ("cone magnification to the first power", "acc += (R / L) * (R / L) * val;", "acc += (R / L) * val;"),
]


def _pin_cases():
    """Every pin test function with one representative argument set."""
    cases = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_") or name == "test_oracle_rejects_bad_arguments":
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if not params:
            cases.append((name, fn, {}))
            continue
        kwargs_list = [{}]
        for m in params:
            names = [n.strip() for n in m.args[0].split(",")]
            new = []
            for kw in kwargs_list:
                for vals in m.args[1]:
                    vals = vals if isinstance(vals, tuple) else (vals,)
                    new.append({**kw, **dict(zip(names, vals))})
            kwargs_list = new
        for kw in kwargs_list:
            cases.append((name, fn, kw))
    return cases


@pytest.mark.parametrize("label,find,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(label, find, repl, tmp_path, monkeypatch):
    src = open(SRC).read()
    assert find in src, f"mutation anchor for {label!r} not found"
    mutated = src.replace(find, repl, 1)
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", str(c_path), "-o",
                    str(so_path), "-lm"], check=True)
    monkeypatch.setattr(oracle, "_lib", oracle.load_library(str(so_path)))
    failed = []
    for name, fn, kw in _pin_cases():
        try:
            fn(**kw)
        except AssertionError:
            failed.append(name)
            break
    assert failed, f"no pin caught the planted mistake {label!r}"
