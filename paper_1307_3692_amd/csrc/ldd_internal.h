// Host-side helpers shared by the library's translation units.
#pragma once

void ldd_set_error(const char* fmt, ...);
