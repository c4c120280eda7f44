"""Device allocation failure through the C ABI: with the device memory held
by a filler allocation, building tables of 65,535 w-planes x 128 sub-cells
(about 2 GB) must fail with SEPW_ERR_OOM (-4), leave nothing half-built, and
the same call must succeed once the memory is free again."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_07152_amd import _lib
    _lib.load()
    return _lib


def test_out_of_memory_is_reported(lib):
    fov = math.radians(2.0)
    args = (64, fov, 1, 128, 65535, -100.0, 100.0)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    left = 1 << 30                      # about half of what the tables need
    filler = torch.empty(free - left, dtype=torch.uint8, device="cuda")
    try:
        with pytest.raises(lib.SepwError) as err:
            lib.Kernels(*args)
        assert err.value.code == -4
    finally:
        del filler
        torch.cuda.empty_cache()
    K = lib.Kernels(*args)
    assert tuple(K.table(0).shape) == (65535, 128, 1)
