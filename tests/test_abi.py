"""CPU checks of the C ABI library: it loads without a GPU and exports every
function that include/krr.h declares.  No compute call is made."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1805_00569_amd import krr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_four_calls():
    names = krr.exported_symbols()
    for n in ("krr_partition", "krr_fit", "krr_predict", "krr_select", "krr_create", "krr_destroy",
              "krr_last_error", "krr_model_free"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(krr.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(krr.LIB_PATH)
    for name in krr.exported_symbols():
        assert hasattr(lib, name), name
    assert set(krr._SIGS) == set(krr.exported_symbols())


def test_struct_layouts_match_header():
    # krr_fit_params: double, double, int32, int32, double, int32, int32, double, double, int32, int32 -> 64 bytes
    assert ctypes.sizeof(krr.FitParams) == 64
    # krr_part_info: 8 x int32 + 4 doubles -> 64 bytes
    assert ctypes.sizeof(krr.PartInfo) == 64
    # krr_server_config: 4 x int32, int64, size_t -> 32 bytes
    assert ctypes.sizeof(krr.ServerConfig) == 32
    # krr_request_info: 4 x int32 + 3 doubles -> 40 bytes
    assert ctypes.sizeof(krr.RequestInfo) == 40
    # krr_serve_stats: 9 x int64 + 5 doubles -> 112 bytes
    assert ctypes.sizeof(krr.ServeStats) == 112


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs gcc and the HIP headers")
def test_struct_layouts_match_compiled_header(tmp_path):
    """Sizes and field offsets of the binding's structures equal what a C
    compiler makes of include/krr.h."""
    structs = {"krr_fit_params": krr.FitParams, "krr_part_info": krr.PartInfo,
               "krr_server_config": krr.ServerConfig, "krr_request_info": krr.RequestInfo,
               "krr_serve_stats": krr.ServeStats}
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "krr.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                          text=True).stdout.split("\n") if line)
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
