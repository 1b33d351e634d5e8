"""MI355X-native CLoD-GS render path (see ``include/clod.h`` for the C ABI)."""
