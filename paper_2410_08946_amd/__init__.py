"""MI355X (gfx950) watershed / waterfall partitioning behind a C ABI.

Python side of libws (include/ws.h): argument marshalling only. Every step of
the hot path runs in the HIP kernels of libws.so; torch supplies device memory
and the current stream. Importing this package does not touch the GPU; the
first call loads libws.so and fails loudly if it has not been built.

Functions named like the C entry points take and return torch tensors:
  ws_gradient(img, sigma, dtype)                  -> uint8/uint16 gradient
  ws_watershed(grad, conn)                         -> int32 canonical labels
  ws_waterfall(labels, grad, conn, NL)             -> (int32 [NL, ...], int64 [NL])
  ws_waterfall_recon(labels, grad, conn, NL)       -> (int32 [NL, ...], int64 [NL]), Alg. 4 + 5
  ws_watershed_stages(grad, conn)                  -> (balanced states, arrows)
  ws_rag(labels, grad, conn)                       -> (a, b, h) region adjacency graph, sorted by (a, b)
  ws_batch([grad, ...], conn, NL)                  -> ([int32 [NL, ...]], [int64 [NL]])
Image tensors are C-contiguous (nx,), (ny, nx) or (nz, ny, nx) with x fastest.
`autotune` picks tile shapes and Step II / III schedules per input class.
"""
from __future__ import annotations

from . import autotune  # noqa: F401
from .binding import (  # noqa: F401
    Context,
    WSError,
    default_context,
    lib_path,
    load_library,
    ws_gradient,
    ws_watershed,
    ws_waterfall,
    ws_waterfall_recon,
    ws_rag,
    ws_watershed_stages,
    ws_batch,
    WS_U8,
    WS_U16,
)
