"""The binding's checks of device buffers (CPU only: every case here is
refused before any pointer reaches the library).

The C ABI takes device buffers as bare pointers whose lengths it cannot
see, so the binding checks each one: a torch tensor on the context's device,
contiguous, of the expected element type and length.  A host array, a CPU
tensor, a strided view, a float32 buffer where float64 is expected, or a
short buffer is refused with ValueError.
"""
import numpy as np
import pytest

torch = pytest.importorskip('torch')

from paper_2311_14106_amd import mdmrg  # noqa: E402


def test_host_arrays_and_cpu_tensors_are_refused():
    with pytest.raises(ValueError, match='torch tensor'):
        mdmrg.device_ptr(np.zeros(8), 0, 8)
    with pytest.raises(ValueError, match='torch tensor'):
        mdmrg.device_ptr(12345, 0, 8)
    with pytest.raises(ValueError, match='cuda:0'):
        mdmrg.device_ptr(torch.zeros(8, dtype=torch.float64), 0, 8)


class _FakeDeviceTensor:
    """Stands in for a device tensor (no GPU here): only the attributes the
    check reads."""

    def __init__(self, n, dtype='torch.float64', contiguous=True, index=0):
        self.is_cuda = True
        self.device = type('dev', (), {'index': index, '__str__': lambda s: f'cuda:{index}'})()
        self.dtype = dtype
        self._n = n
        self._c = contiguous

    def data_ptr(self):
        return 0x1000

    def is_contiguous(self):
        return self._c

    def numel(self):
        return self._n


def test_device_tensor_checks():
    assert mdmrg.device_ptr(_FakeDeviceTensor(8), 0, 8).value == 0x1000
    with pytest.raises(ValueError, match='cuda:0'):
        mdmrg.device_ptr(_FakeDeviceTensor(8, index=1), 0, 8)
    with pytest.raises(ValueError, match='float64'):
        mdmrg.device_ptr(_FakeDeviceTensor(8, dtype='torch.float32'), 0, 8)
    with pytest.raises(ValueError, match='contiguous'):
        mdmrg.device_ptr(_FakeDeviceTensor(8, contiguous=False), 0, 8)
    with pytest.raises(ValueError, match='expected 8 elements, got 7'):
        mdmrg.device_ptr(_FakeDeviceTensor(7), 0, 8)
    # split-form buffers of the grouped GEMM are float32, of any length
    assert mdmrg.device_ptr(_FakeDeviceTensor(5, dtype='torch.float32'), 0, None, 'torch.float32').value == 0x1000
    with pytest.raises(ValueError, match='float32'):
        mdmrg.device_ptr(_FakeDeviceTensor(5), 0, None, 'torch.float32')
