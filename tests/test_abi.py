"""CPU checks of the C ABI library: it loads without a GPU and exports every
function that include/krr.h declares.  No compute call is made."""
import ctypes
import os

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
    # krr_fit_params: double, double, int32, int32, double, int32, int32 -> 40 bytes
    assert ctypes.sizeof(krr.FitParams) == 40
    # krr_part_info: 8 x int32 + double -> 40 bytes
    assert ctypes.sizeof(krr.PartInfo) == 40
    # krr_server_config: 4 x int32, int64, size_t -> 32 bytes
    assert ctypes.sizeof(krr.ServerConfig) == 32
    # krr_request_info: 4 x int32 + 3 doubles -> 40 bytes
    assert ctypes.sizeof(krr.RequestInfo) == 40
    # krr_serve_stats: 8 x int64 + 5 doubles -> 104 bytes
    assert ctypes.sizeof(krr.ServeStats) == 104
