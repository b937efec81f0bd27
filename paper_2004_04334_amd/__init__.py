"""MI355X-native pixel clustering behind a non-blocking acquire/produce boundary."""
