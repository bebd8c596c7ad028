"""A batch of independent cases advanced together (liblbm_axi.so batches).

torch allocates the device pool and the stream; admission, scheduling, the
per-step launches and the hipGraph replays all happen in the library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi


class Batch:
    def __init__(self, pool_bytes: int, max_cases: int = 64, precision: str = "fp32",
                 device="cuda:0", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("Batch needs a HIP device")
        self.device = torch.device(device)
        self.precision = precision
        self.max_cases = max_cases
        self.pool = torch.empty(pool_bytes + 256, dtype=torch.uint8, device=self.device)
        self.pool_ptr = (self.pool.data_ptr() + 255) // 256 * 256
        self.pool_bytes = pool_bytes
        if stream is None:
            stream = torch.cuda.Stream(device=self.device)      # default priority
        self.stream = stream
        with torch.cuda.device(self.device):
            self.handle = abi.lbm_axi_batch_create(self.pool_ptr, pool_bytes, max_cases,
                                                   abi.PRECISIONS[precision], stream.cuda_stream)
        self.specs = {}

    def close(self):
        if getattr(self, "handle", None):
            abi.lbm_axi_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def footprint(spec, precision: str) -> int:
        return abi.lbm_axi_state_bytes(abi.make_params(spec, precision))

    @staticmethod
    def head_bytes(max_cases: int, precision: str) -> int:
        """Bytes at the head of a pool for the case table and the work list."""
        return abi.lbm_axi_batch_reserved_bytes(max_cases, abi.PRECISIONS[precision])

    @classmethod
    def pool_for(cls, specs, precision: str, max_cases: int | None = None) -> int:
        """Pool bytes that hold the head and every case of `specs` at once."""
        n = len(specs) if max_cases is None else max_cases
        return cls.head_bytes(n, precision) + sum(cls.footprint(s, precision) for s in specs)

    def admit(self, spec, nsteps: int):
        """Slot of the admitted case, or None if no slot or pool block is free."""
        phi0 = np.ascontiguousarray(spec.phi0, dtype=np.float64)
        slot = abi.lbm_axi_batch_admit(self.handle, abi.make_params(spec, self.precision), phi0, nsteps)
        if slot is not None:
            self.specs[slot] = spec
        return slot

    def run(self, chunk_steps: int) -> None:
        abi.lbm_axi_batch_run(self.handle, chunk_steps)

    def prepare(self, chunk_steps: int) -> None:
        """Host-side set-up of a run of chunk_steps (work list, graph capture), no launch."""
        abi.lbm_axi_batch_prepare(self.handle, chunk_steps)

    def poll(self):
        return abi.lbm_axi_batch_poll(self.handle)

    def moments(self, slot: int, fields: bool = True):
        spec = self.specs[slot]
        out = {k: np.empty((spec.nr, spec.nz)) for k in ("phi", "rho", "uz", "ur", "p")} if fields else {}
        rc, diag = abi.lbm_axi_batch_moments(self.handle, slot, out.get("phi"), out.get("rho"),
                                             out.get("uz"), out.get("ur"), out.get("p"))
        return out, diag, rc

    def get_state(self, slot: int):
        spec = self.specs[slot]
        f = np.empty((9, spec.nr, spec.nz))
        g = np.empty((9, spec.nr, spec.nz))
        aux = np.empty((3, spec.nr, spec.nz))
        t = abi.lbm_axi_batch_get_state(self.handle, slot, f, g, aux)
        return f, g, aux, t

    def release(self, slot: int) -> None:
        abi.lbm_axi_batch_release(self.handle, slot)
        self.specs.pop(slot, None)

    def set_config(self, tile_r: int = 8, persistent: int = 0, schedule: int = 1, bands: int = 16) -> None:
        abi.lbm_axi_batch_set_config(self.handle, tile_r, persistent, schedule, bands)

    def info(self) -> dict:
        return abi.lbm_axi_batch_info(self.handle)

    def sync(self) -> None:
        abi.lbm_axi_batch_sync(self.handle)
