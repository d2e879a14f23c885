"""The C-ABI library loads, exports every function the header declares, and
lays its structs out as the header says; host-side validation paths that
return before any HIP call are exercised without a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lidar_sim.h")


@pytest.fixture(scope="module")
def binding():
    from paper_2512_05932_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _binding


def _declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lidar_sim_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function(binding):
    lib = binding.load()
    declared = _declared_functions()
    assert declared == sorted(binding.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    # and nothing the header does not declare is exported under the prefix
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = sorted(set(re.findall(r"\b(lidar_sim_[a-z_]+)\b", out)))
    assert exported == declared


def test_struct_layout_matches_header(binding, tmp_path):
    """Compile a probe against the header with gcc and compare sizes and
    offsets with the ctypes mirrors."""
    probe = tmp_path / "probe.c"
    structs = {"lidar_sim_params": binding.lidar_sim_params,
               "lidar_pattern_desc": binding.lidar_pattern_desc,
               "lidar_gbuffer_desc": binding.lidar_gbuffer_desc,
               "lidar_stats": binding.lidar_stats,
               "lidar_pinhole_desc": binding.lidar_pinhole_desc,
               "lidar_batch_info": binding.lidar_batch_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"',
             "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} %zu\\n", sizeof({sname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{sname}.{f} %zu\\n", offsetof({sname}, {f}));')
    lines.append('printf("lidar_echo %zu\\n", sizeof(lidar_echo));')
    lines.append('printf("lidar_beam_info %zu\\n", sizeof(lidar_beam_info));')
    lines.append("return 0; }")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", str(probe), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for sname, cls in structs.items():
        assert int(got[sname]) == C.sizeof(cls), sname
        for f, _ in cls._fields_:
            assert int(got[f"{sname}.{f}"]) == getattr(cls, f).offset, f"{sname}.{f}"
    assert int(got["lidar_echo"]) == binding.ECHO_DTYPE.itemsize
    assert int(got["lidar_beam_info"]) == binding.BEAM_DTYPE.itemsize


class _P:
    n_bins = 512
    max_echoes = 3
    bin_ns = 1.0
    threshold = 1e-6
    emit_power = 1.0
    pulse_fwhm_ns = 4.0
    pulse_trunc_sigmas = 4.0
    ambient_const = 0.0
    sun_irradiance = 0.0
    sun_dir = (0.0, 0.0, 1.0)


@pytest.mark.parametrize("field,value,msg", [
    ("n_bins", 0, "n_bins"), ("n_bins", 9000, "n_bins"), ("max_echoes", 0, "max_echoes"),
    ("max_echoes", 9, "max_echoes"), ("bin_ns", 0.0, "bin_ns"), ("bin_ns", float("nan"), "bin_ns"),
    ("pulse_fwhm_ns", -1.0, "pulse_fwhm_ns"), ("threshold", float("inf"), "threshold"),
    ("emit_power", -1.0, "emit_power"), ("sun_irradiance", -2.0, "sun_irradiance"),
    ("pulse_fwhm_ns", 400.0, "257 taps")])
def test_create_rejects_bad_parameters_without_touching_the_gpu(binding, field, value, msg):
    lib = binding.load()
    p = _P()
    setattr(p, field, value)
    prm = binding.make_params(p)
    h = C.c_void_p()
    rc = lib.lidar_sim_create(C.byref(prm), None, C.byref(h))
    assert rc == binding.LIDAR_E_INVALID
    assert not h.value
    assert msg in lib.lidar_sim_last_error(None).decode()


def test_null_arguments_are_rejected(binding):
    lib = binding.load()
    assert lib.lidar_sim_create(None, None, None) == binding.LIDAR_E_INVALID
    prm = binding.make_params(_P(), flags=64)
    h = C.c_void_p()
    assert lib.lidar_sim_create(C.byref(prm), None, C.byref(h)) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_destroy(None) == binding.LIDAR_OK
    assert lib.lidar_sim_set_pattern(None, None) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_simulate_frame(None, 0) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_read_echoes(None, None, None, None, None, 0) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_get_stats(None, None) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_simulate_batch(None, None, None, 0) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_read_batch(None, 0, None, None, None, None, 0) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_batch_info(None, None) == binding.LIDAR_E_INVALID
    assert lib.lidar_sim_reset_batch(None) == binding.LIDAR_E_INVALID


def _static_args(binding, width, height, flags=0):
    """Descriptors of a frame for lidar_sim_simulate_static whose device
    pointers are placeholders: every call here is rejected before any of
    them is read."""
    import numpy as np
    import scenes
    keep: list = []
    prm = binding.make_params(_P(), flags=flags)
    r = scenes.Raster(width, height, -60.0, 60.0, -20.0, 20.0)
    pat = scenes.Pattern(scenes.PATTERN_GAUSS, np.array([0.0, 1.0]), np.array([0.0, -1.0]),
                         sigma_deg=(0.1, 0.1), trunc_sigmas=3.0)
    pd = binding.pattern_desc(pat, keep)
    fake = 0x1000
    gd = binding.lidar_gbuffer_desc(width, height, width, r.az_min, r.az_max, r.el_min, r.el_max,
                                    *([fake] * 6))
    return prm, pd, gd, keep


def test_static_frame_rejects_frames_beyond_its_scratch(binding):
    """16384 x 2048 pixels need 256 MiB of pixel records: more than the
    static array holds; the call says how much it needed."""
    lib = binding.load()
    prm, pd, gd, keep = _static_args(binding, 16384, 2048)
    fake = C.c_void_p(0x1000)
    rc = lib.lidar_sim_simulate_static(C.byref(prm), C.byref(pd), C.byref(gd), None, fake, fake, fake)
    assert rc == binding.LIDAR_E_INVALID
    msg = lib.lidar_sim_last_error(None).decode()
    assert "bytes of scratch" in msg and str(binding.STATIC_SCRATCH_BYTES) in msg


def test_static_frame_rejects_flags_and_null_outputs(binding):
    lib = binding.load()
    fake = C.c_void_p(0x1000)
    prm, pd, gd, keep = _static_args(binding, 64, 32, flags=binding.LIDAR_KEEP_WAVEFORMS)
    rc = lib.lidar_sim_simulate_static(C.byref(prm), C.byref(pd), C.byref(gd), None, fake, fake, fake)
    assert rc == binding.LIDAR_E_INVALID and "flags" in lib.lidar_sim_last_error(None).decode()
    prm, pd, gd, keep = _static_args(binding, 64, 32)
    rc = lib.lidar_sim_simulate_static(C.byref(prm), C.byref(pd), C.byref(gd), None, None, fake, fake)
    assert rc == binding.LIDAR_E_INVALID and "outputs" in lib.lidar_sim_last_error(None).decode()
    rc = lib.lidar_sim_simulate_static(None, C.byref(pd), C.byref(gd), None, fake, fake, fake)
    assert rc == binding.LIDAR_E_INVALID
