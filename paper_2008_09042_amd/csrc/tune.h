// Plan-time kernel choices with a persistent cache (tune.hip).
#pragma once

#include <functional>
#include <string>

namespace mx {

// The current device's architecture name (e.g. "gfx950:sramecc+:xnack-").
std::string device_arch();
// The choice for `key` (the caller makes the key unique per shape and includes the
// architecture): from this process's memory, else from the tuning file, else measure() on
// the device; measured choices are appended to the tuning file.  The file is
// $MAXWELL_TUNE_CACHE if set (empty: no file), else $HOME/.cache/maxwell/tune.txt; one
// "key = value" line per choice.
int tuned_choice(const std::string& key, const std::function<int()>& measure);
// Choices measured and choices reused (memory or file) since the process started.
void tune_counts(long long* measured, long long* reused);

}  // namespace mx
