// long_lines.hpp -- host entry of the chunked solve for contiguous lines longer
// than one workgroup holds (k_long.hip).
#pragma once

#include "dispatch.hpp"

namespace trid {

// Contiguous lines (inner == 1) longer than one workgroup holds: chunked
// solve through a reduced system of two rows per chunk.  ws must hold
// long_lines_workspace(r) bytes; err receives a message for unsupported shapes.
size_t long_lines_workspace(const LineReq &r);
hipError_t launch_long_lines(const LineReq &r, void *ws, hipStream_t s, std::string *err);

}  // namespace trid
