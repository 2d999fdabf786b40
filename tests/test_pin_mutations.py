"""The pins must catch plausible mistakes in the oracle.  Each case plants one
mistake in a temporary copy of the oracle sources (on the CPU), builds it, and
runs the pin suites (pinhole, LiDAR, learned sensor model, ray walk) against
it; the suite has to fail."""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# (name, file, original text, planted mistake)
MUTANTS = [
    ("sign_of_projective_distance", "oracle_impl.h", "REAL dp = d - zc;", "REAL dp = zc - d;"),
    ("rotation_not_transposed", "oracle_impl.h", "f->R[3 * i + j] = (REAL)T[4 * j + i];",
     "f->R[3 * i + j] = (REAL)T[4 * i + j];"),
    ("translation_sign", "oracle_impl.h", "f->t[i] = (REAL)(-acc);", "f->t[i] = (REAL)(acc);"),
    ("pixel_rounded_to_nearest", "oracle_impl.h", "int32_t i = (int32_t)u;",
     "int32_t i = (int32_t)u; if (u - (REAL)i > (REAL)0.5 && i + 1 < f->width) i += 1;"),
    ("x_and_y_swapped_in_projection", "oracle_impl.h", "REAL u = f->fx * (xc * r) + f->cx;",
     "REAL u = f->fx * (yc * r) + f->cx;"),
    ("principal_point_dropped", "oracle_impl.h", "REAL v = f->fy * (yc * r) + f->cy;",
     "REAL v = f->fy * (yc * r);"),
    ("fx_fy_swapped", "oracle_impl.h", "REAL u = f->fx * (xc * r) + f->cx;",
     "REAL u = f->fy * (xc * r) + f->cx;"),
    ("image_indexed_transposed", "oracle_impl.h",
     "const size_t idx = (size_t)j * (size_t)f->width + (size_t)i;",
     "const size_t idx = (size_t)i * (size_t)f->height + (size_t)j;"),
    ("clamp_instead_of_skip_behind_surface", "oracle_impl.h", "if (!(dp >= -f->eps))\n        return 0;",
     "if (dp < -f->eps)\n        dp = -f->eps;"),
    ("weight_not_capped", "oracle_impl.h", "*W = s < w_max ? s : w_max;", "*W = s;"),
    ("average_drops_old_weight", "oracle_impl.h", "REAL n = *D * *W + x * wm;", "REAL n = *D + x * wm;"),
    ("voxel_centre_missing_half", "oracle_impl.h",
     "/* voxel centre p_L */\n    REAL px = ((REAL)gx + half) * f->vs;",
     "/* voxel centre p_L */\n    REAL px = ((REAL)gx) * f->vs;"),
    ("dropoff_sign", "oracle_impl.h", "w = (f->eps + dp) * f->span_inv;", "w = (f->eps - dp) * f->span_inv;"),
    ("max_range_exclusive", "oracle_impl.h",
     "/* a measurement is valid iff 0 < d <= max range (NaN, Inf, <= 0 fail) */\n    if (!(d > 0 && d <= f->d_max))",
     "/* a measurement is valid iff 0 < d <= max range (NaN, Inf, <= 0 fail) */\n    if (!(d > 0 && d < f->d_max))"),
    ("scan_box_misses_truncation_band", "oracle_impl.h", "double zfar = zmax + (double)f->eps;",
     "double zfar = zmax - (double)f->eps;"),
    ("binary16_rounds_toward_zero", "tsdf_oracle.c", "float r = nearbyintf(ax / q) * q;",
     "float r = truncf(ax / q) * q;"),
    # spherical (LiDAR) path
    ("atan_coefficient_wrong", "tsdf_oracle.c", "p = p * t2 + 0.1999355085f;", "p = p * t2 + 0.1899355085f;"),
    ("atan2_arguments_swapped", "oracle_impl.h", "REAL theta = ATAN2(yc, xc);", "REAL theta = ATAN2(xc, yc);"),
    ("polar_angle_from_minus_z", "oracle_impl.h", "REAL phi = ATAN2(SQRT(xc * xc + yc * yc), zc);",
     "REAL phi = ATAN2(SQRT(xc * xc + yc * yc), -zc);"),
    ("no_azimuth_wrap", "oracle_impl.h", "f->full_circle = (REAL)model[1] >= (REAL)6.28318548f;",
     "f->full_circle = 0;"),
    ("interpolation_weights_swapped", "oracle_impl.h",
     "REAL d = (one - fv) * ((one - fu) * r00 + fu * r10) + fv * ((one - fu) * r01 + fu * r11);",
     "REAL d = (one - fu) * ((one - fv) * r00 + fv * r10) + fu * ((one - fv) * r01 + fv * r11);"),
    ("no_interpolation_guard", "oracle_impl.h", "if (!(mx - mn <= f->interp_diff))", "if (0)"),
    ("lidar_depth_is_z", "oracle_impl.h", "REAL dp = d - rv;", "REAL dp = d - zc;"),
    ("lidar_voxel_centre_missing_half", "oracle_impl.h",
     "one = (REAL)1;\n    REAL px = ((REAL)gx + half) * f->vs;", "one = (REAL)1;\n    REAL px = ((REAL)gx) * f->vs;"),
    # learned sensor model
    ("sm_relu_missing", "sensor_model_impl.h", "h1[k] = ora_round_bf16(a > 0.0f ? a : 0.0f);",
     "h1[k] = ora_round_bf16(a);"),
    ("sm_w1_transposed", "sensor_model_impl.h", "a = fmaf(P[SM_W1 + SM_IN * k + m], x[m], a);",
     "a = fmaf(P[SM_W1 + SM_H * m + k], x[m], a);"),
    ("sm_weight_map_sign", "sensor_model_impl.h", "*w = 0.5f * (o[0] + sqrtf(o[0] * o[0] + 4.0f));",
     "*w = 0.5f * (-o[0] + sqrtf(o[0] * o[0] + 4.0f));"),
    ("sm_truncation_scale", "sensor_model_impl.h", "*e = vs * (1.0f + 7.0f * s);", "*e = vs * (1.0f + 6.0f * s);"),
    ("sm_normal_from_wrong_ray", "sensor_model_impl.h", "const float ax = dr * rxr - dl * rxl,",
     "const float ax = dr * rxr - dl * rxr,"),
    ("sm_patch_not_clipped", "sensor_model_impl.h",
     "v = q - d;\n                            v = v < -0.5f ? -0.5f : (v > 0.5f ? 0.5f : v);",
     "v = q - d;"),
    ("sm_gradient_sign", "sensor_model_impl.h", "gw[f * npx + k] += gD * (x - Dp) / sw;",
     "gw[f * npx + k] += gD * (Dp - x) / sw;"),
    ("sm_pixel_truncation_ignored", "oracle_impl.h", "REAL e = (REAL)f->eps_map[idx];", "REAL e = f->eps;"),
    ("sm_bf16_truncates", "sensor_model_impl.h", "u += 0x7fffu + ((u >> 16) & 1u);", "u += 0u;"),
    # ray-walk allocation
    ("walk_tie_order", "oracle_impl.h",
     "const int ax = (tmax[0] <= tmax[1] && tmax[0] <= tmax[2]) ? 0 : (tmax[1] <= tmax[2] ? 1 : 2);",
     "const int ax = (tmax[2] <= tmax[1] && tmax[2] <= tmax[0]) ? 2 : (tmax[1] <= tmax[0] ? 1 : 0);"),
    ("walk_stops_at_depth", "oracle_impl.h", "REAL te = d + f->eps;", "REAL te = d;"),
    ("walk_through_pixel_corner", "oracle_impl.h", "const REAL a = (((REAL)i + half) - f->cx) / f->fx;",
     "const REAL a = ((REAL)i - f->cx) / f->fx;"),
    ("walk_negative_step_boundary", "oracle_impl.h", "tmax[k] = ((REAL)c[k] * B - o[k]) / dir[k];",
     "tmax[k] = ((REAL)(c[k] - 1) * B - o[k]) / dir[k];"),
    ("beam_at_pixel_edge", "oracle_impl.h",
     "REAL uc = (theta - f->az_start) * f->alpha - half;", "REAL uc = (theta - f->az_start) * f->alpha;"),
]


def run_mutant(fname, orig, mutant):
    """Builds the oracle with one planted mistake and runs the pin suites
    against it; returns (anchor count, pytest return code)."""
    with tempfile.TemporaryDirectory() as tmp:
        for f in ("tsdf_oracle.c", "tsdf_oracle.h", "oracle_impl.h", "sensor_model_impl.h"):
            shutil.copy(os.path.join(ORACLE, f), tmp)
        path = os.path.join(tmp, fname)
        text = open(path).read()
        if text.count(orig) != 1:
            return text.count(orig), None
        open(path, "w").write(text.replace(orig, mutant))
        lib = os.path.join(tmp, "libmutant.so")
        subprocess.run(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                        "-o", lib, os.path.join(tmp, "tsdf_oracle.c"), "-lm"], check=True, cwd=tmp)
        env = dict(os.environ, TSDF_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_lidar.py"),
                            os.path.join(ROOT, "tests", "test_oracle_sensor_model.py"),
                            os.path.join(ROOT, "tests", "test_oracle_dda.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        return 1, r.returncode


@pytest.fixture(scope="module")
def mutant_results():
    """All mutants, run concurrently (each is its own process)."""
    workers = max(1, min(8, (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {m[0]: ex.submit(run_mutant, m[1], m[2], m[3]) for m in MUTANTS}
        return {k: f.result() for k, f in futs.items()}


@pytest.mark.parametrize("name,fname,orig,mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(mutant_results, name, fname, orig, mutant):
    count, rc = mutant_results[name]
    assert count == 1, f"mutation anchor not found once: {orig}"
    assert rc != 0, f"pins did not catch the planted mistake '{name}'"
