"""The sine and cosine of the device code (Helmholtz kernel e^{i kappa r}):
polynomial coefficients in bem_device.h against their construction
(csrc/sincos_minimax.py: Remez exchange on the Taylor tail) and the whole
routine -- Cody-Waite reduction, polynomials, quadrant -- emulated in double
precision against numpy's sin and cos.  No GPU."""
import importlib.util
import pathlib
import re

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1510_07244_amd" / "csrc"


def _generator():
    spec = importlib.util.spec_from_file_location("sincos_minimax", CSRC / "sincos_minimax.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _routine(name):
    """Body of a device function in bem_device.h."""
    text = (CSRC / "bem_device.h").read_text()
    start = text.index(f"void {name}(")
    return text[start:text.index("\n}\n", start)]


def _coefficients(body, var, f32):
    """The Horner coefficients of `var` (highest degree first) as written."""
    num = r"(-?0x[0-9a-f.]+p[-+]?\d+|-?\d+\.\d+)" + ("f" if f32 else "")
    first = re.search(rf"{'float' if f32 else 'double'} {var} = {num};", body).group(1)
    rest = re.findall(rf"{var} = fmaf?\({var}, r2, {num}\);", body)
    conv = lambda x: float.fromhex(x) if "0x" in x else float(x)
    vals = [conv(first)] + [conv(x) for x in rest]
    return vals[::-1]  # lowest degree first


@pytest.mark.parametrize("name,f32", [("sincos_cw", False), ("sincos_cw_f32", True)])
def test_coefficients_are_the_minimax_ones(name, f32):
    gen = _generator()
    body = _routine(name)
    typ = np.float32 if f32 else np.float64
    deg = {("sin", False): 7, ("cos", False): 6, ("sin", True): 3, ("cos", True): 3}
    # sine: relative to sin r; cosine: absolute (r in [-pi/2, pi/2])
    bound = {("sin", False): 6e-18, ("cos", False): 1.4e-17,
             ("sin", True): 9.7e-9, ("cos", True): 5.8e-9}
    for kind, var in (("sin", "ps"), ("cos", "pc")):
        got = _coefficients(body, var, f32)
        if kind == "cos":
            assert got[0] == -0.5
            got = got[1:]  # the fixed -1/2 of cos r = 1 - r^2/2 + r^4 Q(r^2)
        ref, levelled = gen.coefficients(kind, deg[(kind, f32)])
        assert got == [float(typ(c)) for c in ref], kind
        assert levelled <= bound[(kind, f32)]
        assert gen.max_rel_error(kind, [typ(c) for c in got]) <= bound[(kind, f32)], kind


def _fma(a, b, c):
    L = np.longdouble
    return np.float64(L(a) * L(b) + L(c))


def _emulate(x, body):
    """The FP64 routine step by step in double precision (fused
    multiply-adds in long double, rounded once)."""
    ps_c = _coefficients(body, "ps", False)[::-1]
    pc_c = _coefficients(body, "pc", False)[::-1]
    one_over_pi = 0.31830988618379067154
    a, b, c = 3.1415926534682512, 1.2154201012607932e-10, 4.044532497591901e-21
    k = np.rint(x * one_over_pi)
    r = _fma(-k, a, x)
    r = _fma(-k, b, r)
    r = _fma(-k, c, r)
    r2 = r * r
    ps = np.full_like(x, ps_c[0])
    for co in ps_c[1:]:
        ps = _fma(ps, r2, co)
    sr = _fma(r * r2, ps, r)
    pc = np.full_like(x, pc_c[0])
    for co in pc_c[1:]:
        pc = _fma(pc, r2, co)
    cr = _fma(r2, pc, 1.0)
    odd = (k.astype(np.int64) & 1) == 1
    return np.where(odd, -sr, sr), np.where(odd, -cr, cr)


def test_fp64_routine_against_numpy():
    """|kappa r| up to a few hundred covers every workload (kappa <= 8 on
    meshes of diameter 2 to 4); the absolute error stays within 1.5 units in
    the last place of 1 (cos r near r = pi/2 is 1 - r^2/2 + ... with
    cancellation), the sine's relative error near 0 within one."""
    body = _routine("sincos_cw")
    x = np.concatenate([np.linspace(-300.0, 300.0, 400001), np.linspace(-1e-3, 1e-3, 2001),
                        np.pi / 4 * np.arange(-200, 201)])
    s, c = _emulate(x, body)
    assert np.abs(s - np.sin(x)).max() <= 3.4e-16
    assert np.abs(c - np.cos(x)).max() <= 3.4e-16
    tiny = np.abs(x) < 1e-3  # relative accuracy of the sine near 0
    assert np.all(np.abs(s[tiny] - np.sin(x[tiny])) <= 2.3e-16 * np.abs(np.sin(x[tiny])) + 1e-300)
