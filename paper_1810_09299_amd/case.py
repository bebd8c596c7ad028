"""One axisymmetric case on the GPU: torch holds the device block and the
stream; every step of the method runs in liblbm_axi.so."""
from __future__ import annotations

import numpy as np
import torch

from . import abi


class AxiCase:
    """Device-resident case built from a case description (see inputs.CaseSpec).

    The device block is a torch uint8 tensor owned by this object; the library
    works on torch's current stream of `device` unless `stream` is given.
    """

    def __init__(self, spec, precision: str = "fp64", device="cuda:0", stream=None, phi0=None):
        if not torch.cuda.is_available():
            raise RuntimeError("AxiCase needs a HIP device")
        self.spec = spec
        self.precision = precision
        self.device = torch.device(device)
        self.nr, self.nz = int(spec.nr), int(spec.nz)
        self.params = abi.make_params(spec, precision)
        nbytes = abi.lbm_axi_state_bytes(self.params)
        if nbytes == 0:
            raise abi.LbmAxiError(abi.LBM_AXI_EINVAL, "lbm_axi_state_bytes")
        self.nbytes = nbytes
        self.block = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.block.data_ptr()
        self.dev_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        phi0 = spec.phi0 if phi0 is None else phi0
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(self.nr, self.nz)
        with torch.cuda.device(self.device):
            self.handle = abi.lbm_axi_init(self.params, self.dev_ptr, nbytes, phi0,
                                           self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            abi.lbm_axi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return abi.lbm_axi_time(self.handle)

    def step(self, n: int = 1) -> None:
        abi.lbm_axi_step(self.handle, n)

    def set_tile(self, tile_r: int) -> None:
        abi.lbm_axi_set_tile(self.handle, tile_r)

    def moments(self, fields: bool = True):
        """(fields dict of float64 (nr, nz) arrays, diagnostics dict, return code)."""
        out = {k: np.empty((self.nr, self.nz)) for k in ("phi", "rho", "uz", "ur", "p")} if fields else {}
        rc, diag = abi.lbm_axi_moments(self.handle, out.get("phi"), out.get("rho"), out.get("uz"),
                                       out.get("ur"), out.get("p"))
        return out, diag, rc

    def diagnostics(self) -> dict:
        return self.moments(fields=False)[1]

    def get_state(self):
        f = np.empty((9, self.nr, self.nz))
        g = np.empty((9, self.nr, self.nz))
        aux = np.empty((3, self.nr, self.nz))
        t = abi.lbm_axi_get_state(self.handle, f, g, aux)
        return f, g, aux, t

    def set_state(self, f, g, aux, t: int = 0) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        aux = np.ascontiguousarray(aux, dtype=np.float64)
        abi.lbm_axi_set_state(self.handle, f, g, aux, t)
