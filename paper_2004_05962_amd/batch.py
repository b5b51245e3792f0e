"""Batched forward + adjoint of many volumes in persistent launches (one HIP graph).

Thin owner of a ``bsi_batch`` plan: create (geometry), bind (device buffers),
tune (schedule of seven knobs chosen by timing, persisted in BSI_TUNE_CACHE), capture, launch.
"""
from . import _lib


class BatchPlan:
    def __init__(self, dims_list, spacing_list):
        self.dims = [tuple(int(v) for v in d) for d in dims_list]
        self.spacing = [tuple(int(v) for v in s) for s in spacing_list]
        self._plan = _lib.bsi_batch_create(self.dims, self.spacing)
        self._bound = None

    def bind(self, grids=None, fields=None, dfields=None, grid_grads=None):
        _lib.bsi_batch_bind(self._plan, grids, fields, dfields, grid_grads)
        self._bound = (grids, fields, dfields, grid_grads)  # keep the tensors alive

    def tune(self, stream=None):
        _lib.bsi_batch_tune(self._plan, stream)
        return self.config()

    def config(self):
        return _lib.bsi_batch_config(self._plan)

    def describe(self):
        return _lib.bsi_batch_describe(self._plan)

    def run(self, stream=None):
        _lib.bsi_batch_run(self._plan, stream)

    def run_separate(self, stream=None):
        _lib.bsi_batch_run_separate(self._plan, stream)

    def capture(self, stream=None):
        _lib.bsi_batch_capture(self._plan, stream)

    def launch(self, stream=None):
        _lib.bsi_batch_launch(self._plan, stream)

    def close(self):
        if self._plan:
            _lib.bsi_batch_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
