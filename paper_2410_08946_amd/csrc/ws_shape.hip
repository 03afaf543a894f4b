// ws_shape.hip -- the watershed tile kernels of one tile shape. The build
// compiles this file once per shape id (-DWS_SHAPE=<id>, see TileShape in
// ws_device.h), so that the shapes' kernels compile in parallel.
#include "ws_tiles.h"

#ifndef WS_SHAPE
#error "WS_SHAPE (a tile shape id) must be defined"
#endif

namespace wsk {
template struct WsShape<WS_SHAPE>;
}  // namespace wsk
